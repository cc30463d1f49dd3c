// Section kernels for CDNA4 (gfx950).
//
// A section (section 2: one data-parallel loop) reads some fields of each
// record -- of the record itself (direct) or of d neighbour records named by
// an index array (gather) -- and writes one or two fields of the record.
// Whatever the layout, field f of record r sits at
//   base_g + (r >> logT) * T*S_g + p_f*T + (r & (T-1)) * e_f,
// so a kernel is generic over layouts through five numbers per field and the
// layout decides the memory traffic: consecutive lanes read consecutive
// records, which is a dense 256-byte run per field in SoA and in T >= 64
// tiles, and a strided walk over whole records in interleaved groups.
// One lane owns one record.  All terms are read before any write, in the
// order the section's definition fixes, and every floating-point step uses
// the explicitly rounded intrinsics so that no multiply-add is fused.
#include <algorithm>
#include <cstdlib>
#include <map>
#include <mutex>

#include "adha_impl.h"

namespace adha {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

struct SField {
  uint64_t base;
  uint32_t TS;    // T * S_g
  uint32_t pT;    // p_f * T
  uint32_t logT;
  uint32_t e;     // 1, 2, 4 or 8
  uint32_t dt;
  uint32_t al;    // 1: every address of the field is a multiple of 4
};

struct SectionArgs {
  uint8_t *buf;
  const int32_t *idx;
  uint32_t *err;
  int64_t n;
  uint32_t degree, n_read, n_write, op;
  SField rd[ADHA_MAX_READ];
  SField wr[ADHA_MAX_WRITE];
  // stencils: neighbours at grid offsets (x, y, z) instead of idx
  uint32_t stencil, nx, ny, nz;
  // r / nx and r / ny for r < 2^31 as (r * m) >> s (m < 2^32, set at launch)
  uint32_t mx, sx, my, sy;
  int32_t off[ADHA_MAX_DEGREE][3];
  int32_t lin[ADHA_MAX_DEGREE];  // the same offsets as record-index steps
};

// Neighbour j of record i: from the index array, or for a stencil the
// record at the grid offset (-1 when outside the grid).
struct Neighbours {
  const int32_t *row = nullptr;
  int32_t x = 0, y = 0, z = 0, i = 0;
  __device__ __forceinline__ Neighbours(const SectionArgs &a, uint64_t rec) {
    if (a.stencil) {
      i = (int32_t)rec;
      x = i % (int32_t)a.nx;
      const int32_t t = i / (int32_t)a.nx;
      y = t % (int32_t)a.ny;
      z = t / (int32_t)a.ny;
    } else {
      row = a.idx + rec * (uint64_t)a.degree;
    }
  }
  __device__ __forceinline__ int32_t get(const SectionArgs &a, int j) const {
    if (!a.stencil) return row[j];
    const int32_t xx = x + a.off[j][0], yy = y + a.off[j][1], zz = z + a.off[j][2];
    const bool in = xx >= 0 && xx < (int32_t)a.nx && yy >= 0 && yy < (int32_t)a.ny && zz >= 0 && zz < (int32_t)a.nz;
    return in ? i + a.lin[j] : -1;
  }
};

__device__ __forceinline__ uint64_t faddr(const SField &F, uint64_t r) {
  return F.base + (r >> F.logT) * F.TS + F.pT + (r & ((1ull << F.logT) - 1)) * F.e;
}

// A field of any width at any address (a 1- or 2-byte field, or a wider one
// placed after narrow fields in an interleaved group), zero-extended: the
// one to three dwords that hold its bytes are loaded and funnel-shifted.
// A dword the field does not reach is replaced by the one before it, so no
// branch depends on the field's width or offset and every load is a dword
// holding a byte of the field.  Such a dword lies inside the field's group
// region, whose base and size are multiples of 256, so it is inside the
// buffer.  Bytes of other fields in those dwords are discarded.  (Loading
// only the dwords a field can reach, by a branch on the field, measured
// slower: the branches split the batches of loads.)
// W8 = false: no field of the section is 8 bytes wide, so the third dword
// is never needed and not loaded.
template <bool W8 = true>
__device__ __forceinline__ uint64_t load_span(const uint8_t *buf, uint32_t e, uint64_t at) {
  const uint32_t *q = reinterpret_cast<const uint32_t *>(buf + (at & ~3ull));
  const uint32_t o = (uint32_t)at & 3u, end = o + e;
  const uint32_t w0 = q[0];
  const uint32_t w1 = q[end > 4 ? 1 : 0];
  const uint32_t lo = __builtin_amdgcn_alignbit(w1, w0, 8 * o);  // bytes o..o+3 of w1:w0
  if constexpr (!W8) return e >= 4 ? lo : lo & ((1u << (8 * e)) - 1u);
  const uint32_t w2 = q[end > 8 ? 2 : (end > 4 ? 1 : 0)];
  const uint32_t hi = __builtin_amdgcn_alignbit(w2, w1, 8 * o);
  const uint32_t mask = e >= 4 ? ~0u : (1u << (8 * e)) - 1u;
  return (uint64_t)(lo & mask) | ((uint64_t)(e == 8 ? hi : 0u) << 32);
}

__device__ __forceinline__ uint64_t load_any(const uint8_t *buf, const SField &F, uint64_t r) {
  return load_span(buf, F.e, faddr(F, r));
}

// The raw words of up to N terms.  Loads only fill registers; the terms are
// assembled afterwards (word() below), so no arithmetic sits between one
// load and the next and all of them are in flight together.  W8: some term
// is 8 bytes wide, so a second word is loaded per term -- for a 4-byte term
// that second load reads the same word again and stays inside the field.
template <int N, bool W8, bool SUB = false>
struct Words {
  uint32_t lo[N];
  uint32_t hi[W8 || SUB ? N : 1];
  __device__ __forceinline__ void load(int q, const uint8_t *buf, const SField &F, uint64_t r) {
    if constexpr (SUB) {  // any width, any alignment
      const uint64_t v = load_any(buf, F, r);
      lo[q] = (uint32_t)v;
      hi[q] = (uint32_t)(v >> 32);
      return;
    }
    const uint32_t *p = reinterpret_cast<const uint32_t *>(buf + faddr(F, r));
    lo[q] = p[0];
    if constexpr (W8) hi[q] = p[F.e >> 3];
  }
  // SUB: the field's element at byte offset off (any width, any alignment)
  __device__ __forceinline__ void load_off(int q, const uint8_t *buf, const SField &F, uint32_t off) {
    const uint64_t v = load_span<W8>(buf, F.e, off);
    lo[q] = (uint32_t)v;
    hi[q] = (uint32_t)(v >> 32);
  }
  __device__ __forceinline__ void load_at(int q, const uint8_t *at, const SField &F) {
    const uint32_t *p = reinterpret_cast<const uint32_t *>(at);
    lo[q] = p[0];
    if constexpr (W8) hi[q] = p[F.e >> 3];
  }
  __device__ __forceinline__ uint64_t term(int q, const SField &F) const {
    if constexpr (SUB) return (uint64_t)lo[q] | ((uint64_t)hi[q] << 32);
    if constexpr (W8) return (uint64_t)lo[q] | ((uint64_t)(F.e == 8 ? hi[q] : 0u) << 32);
    return lo[q];
  }
};

// One term as a single value.  Used by the gathers: there the loads of one
// neighbour's fields complete one after another, so when several fields
// share a memory line (an interleaved group), the later ones hit the line
// the first one brought in instead of each missing on it at the same time
// (measured: batching them made all-AoS gathers 17% slower, with no gain
// on SoA).
__device__ __forceinline__ uint64_t load_term(const uint8_t *buf, const SField &F, uint64_t r) {
  const uint32_t *p = reinterpret_cast<const uint32_t *>(buf + faddr(F, r));
  if (F.e == 4) return p[0];
  return (uint64_t)p[0] | ((uint64_t)p[1] << 32);
}

__device__ __forceinline__ uint32_t load_word(const uint8_t *buf, const SField &F, uint64_t r) {
  return *reinterpret_cast<const uint32_t *>(buf + faddr(F, r));
}

// The value of an integer term (its element bytes zero-extended in b).
__device__ __forceinline__ int64_t int_value(uint32_t dt, uint64_t b) {
  switch (dt) {
    case ADHA_I32: return (int32_t)(uint32_t)b;
    case ADHA_I16: return (int16_t)(uint16_t)b;
    case ADHA_U32: return (uint32_t)b;
    case ADHA_U16: return (uint16_t)b;
    default: return (uint8_t)b;
  }
}

__device__ __forceinline__ float to_f32(uint32_t dt, uint64_t b) {
  if (dt == ADHA_F32) return __uint_as_float((uint32_t)b);
  if (dt == ADHA_I32) return __int2float_rn((int32_t)(uint32_t)b);
  if (dt == ADHA_F64) return __double2float_rn(__longlong_as_double((long long)b));
  if (dt == ADHA_U32) return __uint2float_rn((uint32_t)b);
  return __int2float_rn((int32_t)int_value(dt, b));  // U16, I16, U8: exact
}

__device__ __forceinline__ double to_f64(uint32_t dt, uint64_t b) {
  if (dt == ADHA_F32) return (double)__uint_as_float((uint32_t)b);
  if (dt == ADHA_F64) return __longlong_as_double((long long)b);
  return (double)int_value(dt, b);  // exact for every integer type
}

__device__ __forceinline__ uint32_t bits32(uint32_t dt, uint64_t b) {
  if (dt == ADHA_F64) return (uint32_t)b ^ (uint32_t)(b >> 32);
  if (dt == ADHA_F32) return (uint32_t)b;
  return (uint32_t)(uint64_t)int_value(dt, b);
}

struct Acc {
  float f;
  double d;
  uint32_t u;
};

// Fold one term into write k's accumulator (GEN and SUM).
__device__ __forceinline__ void fold(Acc &a, uint32_t k, uint32_t wdt, uint32_t tdt, uint64_t t) {
  if (wdt == ADHA_F32) {
    const float v = to_f32(tdt, t);
    a.f = k == 0 ? __fadd_rn(a.f, v) : __fadd_rn(__fmul_rn(a.f, 0.5f), v);
  } else if (wdt == ADHA_F64) {
    const double v = to_f64(tdt, t);
    a.d = k == 0 ? __dadd_rn(a.d, v) : __dadd_rn(__dmul_rn(a.d, 0.5), v);
  } else {
    const uint32_t u = bits32(tdt, t);
    a.u = k == 0 ? a.u + u : (a.u ^ u) * 16777619u;
  }
}

// Little-endian bytes of v, one store each (a field that is narrower than 4
// bytes or not 4-byte aligned).
__device__ __forceinline__ void store_bytes(uint8_t *at, uint64_t v, uint32_t e) {
  for (uint32_t q = 0; q < e; ++q) at[q] = (uint8_t)(v >> (8 * q));
}

// Each type stores from its own branch: the three-way choice of the element
// bits ahead of one shared store was compiled (for the generic section
// kernel) with the integer branch's value left undefined, so no value is
// merged across the branches here.  An integer field keeps the low bytes of
// the fold.
__device__ __forceinline__ void store_acc(uint8_t *buf, const SField &W, uint64_t r, const Acc &a) {
  uint8_t *at = buf + faddr(W, r);
  if (W.al) {
    uint32_t *p = reinterpret_cast<uint32_t *>(at);
    if (W.dt == ADHA_F32) {
      p[0] = __float_as_uint(a.f);
    } else if (W.dt == ADHA_F64) {
      const uint64_t b = (uint64_t)__double_as_longlong(a.d);
      p[0] = (uint32_t)b;
      p[1] = (uint32_t)(b >> 32);
    } else {
      p[0] = a.u;
    }
  } else if (W.dt == ADHA_F32) {
    store_bytes(at, __float_as_uint(a.f), 4);
  } else if (W.dt == ADHA_F64) {
    store_bytes(at, (uint64_t)__double_as_longlong(a.d), 8);
  } else if (W.e == 2 && ((W.TS | W.pT) & 1u) == 0) {
    *reinterpret_cast<uint16_t *>(at) = (uint16_t)a.u;  // a 2-byte field at an even address
  } else {
    store_bytes(at, a.u, W.e);
  }
}

// The GEN / SUM fold specialised on the write types (WT0, WT1: 0 an F32
// write, 1 F64, 2 an integer fold; WT1 = 3: one write).  Every term is
// converted by computing each candidate conversion and keeping the one its
// type names, so no branch depends on a field's type; the conversions are
// those of to_f32, to_f64 and bits32 (nearest even).  lo, hi: the term's
// element bytes, zero-extended (hi only for an 8-byte term, W8).  NAR: terms
// may also be U16, I16 or U8, and write fields narrow or unaligned.
template <int WT0, int WT1, bool W8, bool NAR>
struct MixFold {
  float f0 = 0.0f, f1 = 0.0f;
  double d0 = 0.0, d1 = 0.0;
  uint32_t u0 = 0u, u1 = 0u;
  // take = false leaves the accumulators as they are
  __device__ __forceinline__ void add(uint32_t dt, uint32_t lo, uint32_t hi, bool take) {
    const double dbits = __longlong_as_double((long long)(((uint64_t)(W8 ? hi : 0u) << 32) | lo));
    const int32_t s16 = (int32_t)(int16_t)(uint16_t)lo;
    if constexpr (WT0 == 0 || WT1 == 0) {
      // I32, U16 and U8 (zero-extended) convert as the int32 lo
      const float c_f = __uint_as_float(lo), c_i = __int2float_rn((int32_t)lo), c_u = __uint2float_rn(lo);
      const float c_d = W8 ? __double2float_rn(dbits) : 0.0f;
      float v = dt == ADHA_F32 ? c_f : dt == ADHA_U32 ? c_u : dt == ADHA_F64 ? c_d : c_i;
      if constexpr (NAR) v = dt == ADHA_I16 ? __int2float_rn(s16) : v;
      if constexpr (WT0 == 0) f0 = take ? __fadd_rn(f0, v) : f0;
      if constexpr (WT1 == 0) f1 = take ? __fadd_rn(__fmul_rn(f1, 0.5f), v) : f1;
    }
    if constexpr (WT0 == 1 || WT1 == 1) {
      const double c_f = (double)__uint_as_float(lo), c_i = (double)(int32_t)lo, c_u = (double)lo;
      double v = dt == ADHA_F32 ? c_f : dt == ADHA_U32 ? c_u : dt == ADHA_F64 ? dbits : c_i;
      if constexpr (NAR) v = dt == ADHA_I16 ? (double)s16 : v;
      if constexpr (WT0 == 1) d0 = take ? __dadd_rn(d0, v) : d0;
      if constexpr (WT1 == 1) d1 = take ? __dadd_rn(__dmul_rn(d1, 0.5), v) : d1;
    }
    if constexpr (WT0 == 2 || WT1 == 2) {
      // an F32, I32, U32, U16 or U8 term is its own (zero-extended) bits
      uint32_t v = dt == ADHA_F64 ? lo ^ hi : lo;
      if constexpr (NAR) v = dt == ADHA_I16 ? (uint32_t)s16 : v;
      if constexpr (WT0 == 2) u0 = take ? u0 + v : u0;
      if constexpr (WT1 == 2) u1 = take ? (u1 ^ v) * 16777619u : u1;
    }
  }
  template <int WT>
  __device__ __forceinline__ static void put1(uint8_t *buf, const SField &W, uint64_t i, float f, double d,
                                              uint32_t u) {
    uint8_t *at = buf + faddr(W, i);
    uint32_t *p = reinterpret_cast<uint32_t *>(at);
    const uint64_t db = (uint64_t)__double_as_longlong(d);
    if (!NAR || W.al) {
      if constexpr (WT == 0) {
        p[0] = __float_as_uint(f);
      } else if constexpr (WT == 1) {
        p[0] = (uint32_t)db;
        p[1] = (uint32_t)(db >> 32);
      } else {
        p[0] = u;
      }
    } else if constexpr (WT == 0) {
      store_bytes(at, __float_as_uint(f), 4);
    } else if constexpr (WT == 1) {
      store_bytes(at, db, 8);
    } else if (W.e == 2 && ((W.TS | W.pT) & 1u) == 0) {
      *reinterpret_cast<uint16_t *>(at) = (uint16_t)u;  // a 2-byte field at an even address
    } else {
      store_bytes(at, u, W.e);  // an integer field keeps the low bytes of the fold
    }
  }
  __device__ __forceinline__ void put(uint8_t *buf, const SectionArgs &a, uint64_t i) const {
    put1<WT0>(buf, a.wr[0], i, f0, d0, u0);
    if constexpr (WT1 != 3) put1<WT1>(buf, a.wr[1], i, f1, d1, u1);
  }
};

// DG = 0: direct section; otherwise a gather of at most DG neighbours.
// MAXR: bound on the number of read fields (loads are unrolled to it).
// W8: some read field is 8 bytes wide.
// SUB: some field is narrower than 4 bytes or not 4-byte aligned, so every
// field is read through load_any.
template <int OP, int DG, int MAXR, bool W8, bool SUB = false>
__global__ __launch_bounds__(256) void section_kernel(const SectionArgs a) {
  const uint64_t i = (uint64_t)blockIdx.x * 256u + threadIdx.x;
  if (i >= (uint64_t)a.n) return;
  const uint32_t nr = a.n_read, nw = a.n_write;
  Acc acc[2];
  acc[0] = acc[1] = Acc{0.0f, 0.0, 0u};

  if constexpr (DG == 0) {
    Words<MAXR, W8, SUB> w;
#pragma unroll
    for (int q = 0; q < MAXR; ++q)
      if (q < (int)nr) w.load(q, a.buf, a.rd[q], i);
    uint64_t tv[MAXR];
#pragma unroll
    for (int q = 0; q < MAXR; ++q) tv[q] = q < (int)nr ? w.term(q, a.rd[q]) : 0;
    if constexpr (OP == ADHA_OP_GEN || OP == ADHA_OP_SUM) {
#pragma unroll
      for (int q = 0; q < MAXR; ++q)
        if (q < (int)nr) {
          fold(acc[0], 0, a.wr[0].dt, a.rd[q].dt, tv[q]);
          if (nw > 1) fold(acc[1], 1, a.wr[1].dt, a.rd[q].dt, tv[q]);
        }
    } else {
      const uint32_t wdt = a.wr[0].dt;
      if (wdt == ADHA_F32) {
        const float x = to_f32(a.rd[0].dt, tv[0]), y = to_f32(a.rd[1].dt, tv[1]);
        if constexpr (OP == ADHA_OP_MULADD3)
          acc[0].f = __fadd_rn(__fmul_rn(x, y), to_f32(a.rd[2].dt, tv[2]));
        else
          acc[0].f = __fsub_rn(x, y);
      } else {
        const double x = to_f64(a.rd[0].dt, tv[0]), y = to_f64(a.rd[1].dt, tv[1]);
        if constexpr (OP == ADHA_OP_MULADD3)
          acc[0].d = __dadd_rn(__dmul_rn(x, y), to_f64(a.rd[2].dt, tv[2]));
        else
          acc[0].d = __dsub_rn(x, y);
      }
    }
  } else {
    // Neighbours are taken in batches of NB with all of a batch's field loads
    // in flight together; the next batch's indices are loaded before the
    // current batch's fields, so the two round trips overlap.  Terms are
    // folded in neighbour order.
    constexpr int NB = MAXR >= 32 ? 1 : 32 / MAXR;
    const int deg = (int)a.degree;
    const Neighbours nb(a, i);
    int32_t cur[NB], nxt[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) cur[b] = b < deg ? nb.get(a, b) : 0;
    bool bad = false;
    for (int j0 = 0; j0 < deg; j0 += NB) {
#pragma unroll
      for (int b = 0; b < NB; ++b) nxt[b] = j0 + NB + b < deg ? nb.get(a, j0 + NB + b) : 0;
      uint64_t t[NB][MAXR];
      bool ok[NB];
#pragma unroll
      for (int b = 0; b < NB; ++b) {
        const bool live = j0 + b < deg;
        ok[b] = live && cur[b] >= 0 && (int64_t)cur[b] < a.n;
        bad |= live && !ok[b] && !a.stencil;   // a stencil neighbour off the grid is no error
#pragma unroll
        for (int q = 0; q < MAXR; ++q)
          if (q < (int)nr) {
            if constexpr (SUB) t[b][q] = ok[b] ? load_any(a.buf, a.rd[q], (uint64_t)cur[b]) : 0;
            else t[b][q] = ok[b] ? load_term(a.buf, a.rd[q], (uint64_t)cur[b]) : 0;
          }
      }
#pragma unroll
      for (int b = 0; b < NB; ++b)
        if (ok[b]) {
#pragma unroll
          for (int q = 0; q < MAXR; ++q)
            if (q < (int)nr) {
              fold(acc[0], 0, a.wr[0].dt, a.rd[q].dt, t[b][q]);
              if (nw > 1) fold(acc[1], 1, a.wr[1].dt, a.rd[q].dt, t[b][q]);
            }
        }
#pragma unroll
      for (int b = 0; b < NB; ++b) cur[b] = nxt[b];
    }
    if (bad) atomicOr(a.err, 1u);
  }
  store_acc(a.buf, a.wr[0], i, acc[0]);
  if (nw > 1) store_acc(a.buf, a.wr[1], i, acc[1]);
}

// Direct GEN / SUM sections whose read and write fields are all F32: the
// generic kernel's fold branches on the field types per term, which costs
// tens of scalar instructions per term and bounds the loop by instruction
// issue; here the fold is straight-line.  Loads are not guarded: descriptors
// past the read count are zero, so those slots load the buffer's first word
// and are never folded.  LIN: every read field sits in a group with T = 1
// and the layout fits in 4 GiB, so a field's offset is base + p + r*S in 32
// bits.
// Direct GEN / SUM sections over F32, F64, I32 and U32 fields at 4-byte
// aligned addresses, not all F32 (NAR = false), or with some field narrow
// or unaligned (NAR = true: every field through load_any, stores that fit
// each write field).  The generic kernel's fold branches on the write type
// and the term type of every term, tens of scalar instructions per term;
// here the fold is MixFold, specialised on the write types and converting
// terms by selects.
// RPT records per thread, one per 256-record chunk of the workgroup's RPT
// chunks, all their loads issued before any fold: a section with few fields
// streams few bytes per record, and one record per thread leaves too few
// bytes in flight.
template <int MAXR, bool W8, int WT0, int WT1, int RPT, bool NAR = false>
__global__ __launch_bounds__(256) void direct_mixed_kernel(const SectionArgs a) {
  const uint32_t nr = a.n_read;
  Words<MAXR, W8, NAR> w[RPT];
  uint64_t rec[RPT];
  bool live[RPT];
#pragma unroll
  for (int r = 0; r < RPT; ++r) {
    rec[r] = ((uint64_t)blockIdx.x * RPT + r) * 256u + threadIdx.x;
    live[r] = rec[r] < (uint64_t)a.n;
    const uint64_t rr = live[r] ? rec[r] : 0;  // past N: record 0, nothing stored
#pragma unroll
    for (int q = 0; q < MAXR; ++q)
      if (q < (int)nr) w[r].load(q, a.buf, a.rd[q], rr);
  }
#pragma unroll
  for (int r = 0; r < RPT; ++r) {
    if (!live[r]) continue;
    MixFold<WT0, WT1, W8 || NAR, NAR> m;
#pragma unroll
    for (int q = 0; q < MAXR; ++q)
      if (q < (int)nr) m.add(a.rd[q].dt, w[r].lo[q], W8 || NAR ? w[r].hi[q] : 0u, true);
    m.put(a.buf, a, rec[r]);
  }
}

template <int MAXR, bool W8, int WT0, bool NAR>
static void launch_direct_mixed_w1(int wt1, const SectionArgs &a, hipStream_t st) {
  // 4 records per thread for up to 4 reads, else 1
  constexpr int RPT = MAXR <= 4 ? 4 : 1;
  const dim3 grid((uint32_t)(((uint64_t)a.n + 256ull * RPT - 1) / (256ull * RPT)));
  switch (wt1) {
    case 0: hipLaunchKernelGGL((direct_mixed_kernel<MAXR, W8, WT0, 0, RPT, NAR>), grid, dim3(256), 0, st, a); break;
    case 1: hipLaunchKernelGGL((direct_mixed_kernel<MAXR, W8, WT0, 1, RPT, NAR>), grid, dim3(256), 0, st, a); break;
    case 2: hipLaunchKernelGGL((direct_mixed_kernel<MAXR, W8, WT0, 2, RPT, NAR>), grid, dim3(256), 0, st, a); break;
    default: hipLaunchKernelGGL((direct_mixed_kernel<MAXR, W8, WT0, 3, RPT, NAR>), grid, dim3(256), 0, st, a); break;
  }
}

template <int MAXR, bool W8, bool NAR = false>
static void launch_direct_mixed_w0(int wt0, int wt1, const SectionArgs &a, hipStream_t st) {
  if (wt0 == 0) launch_direct_mixed_w1<MAXR, W8, 0, NAR>(wt1, a, st);
  else if (wt0 == 1) launch_direct_mixed_w1<MAXR, W8, 1, NAR>(wt1, a, st);
  else launch_direct_mixed_w1<MAXR, W8, 2, NAR>(wt1, a, st);
}

// RPT records per thread, one per 256-record chunk of the workgroup's RPT
// chunks, every load issued before any fold (a few fields per record leave
// too few bytes in flight at one record per thread).
template <int MAXR, bool LIN, int RPT>
__global__ __launch_bounds__(256) void direct_f32_kernel(const SectionArgs a) {
  const uint32_t nr = a.n_read, nw = a.n_write;
  uint32_t w[RPT][MAXR];
  uint64_t rec[RPT];
#pragma unroll
  for (int r = 0; r < RPT; ++r) {
    rec[r] = ((uint64_t)blockIdx.x * RPT + r) * 256u + threadIdx.x;
    const uint64_t i = rec[r] < (uint64_t)a.n ? rec[r] : 0;  // past N: record 0, nothing stored
#pragma unroll
    for (int q = 0; q < MAXR; ++q) {
      const SField &F = a.rd[q];
      if constexpr (LIN) {
        const uint32_t off = (uint32_t)F.base + F.pT + (uint32_t)i * F.TS;
        w[r][q] = *reinterpret_cast<const uint32_t *>(a.buf + off);
      } else {
        w[r][q] = *reinterpret_cast<const uint32_t *>(a.buf + faddr(F, i));
      }
    }
  }
#pragma unroll
  for (int r = 0; r < RPT; ++r) {
    if (rec[r] >= (uint64_t)a.n) continue;
    float acc0 = 0.0f, acc1 = 0.0f;
#pragma unroll
    for (int q = 0; q < MAXR; ++q)
      if (q < (int)nr) {
        const float v = __uint_as_float(w[r][q]);
        acc0 = __fadd_rn(acc0, v);
        if (nw > 1) acc1 = __fadd_rn(__fmul_rn(acc1, 0.5f), v);
      }
    *reinterpret_cast<uint32_t *>(a.buf + faddr(a.wr[0], rec[r])) = __float_as_uint(acc0);
    if (nw > 1) *reinterpret_cast<uint32_t *>(a.buf + faddr(a.wr[1], rec[r])) = __float_as_uint(acc1);
  }
}

// Workgroups go to the chip's 8 XCDs round-robin (workgroup b to XCD b mod
// 8), and each XCD has an L2 of its own.  Block xcd_block(b, G) gives XCD x
// one contiguous range of the G blocks, so that the records a neighbour at a
// grid offset needs were brought into that XCD's L2 by its own recent
// blocks.  A bijection of [0, G) for any G.
__device__ __forceinline__ uint32_t xcd_block(uint32_t b, uint32_t G) {
  const uint32_t x = b & 7u, q = G >> 3, r = G & 7u;
  return x * q + min(x, r) + (b >> 3);
}

// Stencil sections: the neighbours are the record's grid neighbourhood, so
// consecutive lanes read consecutive records at every offset and most loads
// hit lines other lanes or offsets just brought in.  Here all the loads of
// a batch of neighbours are issued together (no index array, no arithmetic
// between the loads); an off-grid neighbour loads the record itself and is
// dropped.  Terms are folded in neighbour order.
//
// A stencil makes many terms per byte it streams, so the per-term work is
// what bounds it rather than HBM:
//  * LIN: every read field sits in a group with T = 1, where a field's
//    address is linear in the record index (base + r*S + p), so a
//    neighbour's field is the record's own field offset plus the offset's
//    record step times S.  The launch takes this form only when the layout
//    fits in 4 GiB, every such product in 31 bits, and steps and S in 24
//    signed bits, so offsets are 32-bit and one neighbour's field costs one
//    24-bit multiply-add;
//  * F32: every read and write field is F32 (W8 is then false), and the
//    fold is straight-line code: an off-grid neighbour's term is computed
//    and not selected, instead of branching on the field types per term
//    (the generic fold spends tens of scalar instructions per term on them);
//  * EXACT: the section reads exactly MAXR fields, so no load is guarded;
//  * DEG > 0: the stencil has exactly DEG neighbours, taken in one batch
//    (a 7-point stencil in batches of 8 would load an eighth, unused one);
//  * ROW: nx is a multiple of 64, so the 64 records of a wave lie in one
//    grid row and share y and z: those two tests are scalar, and only x is
//    tested per lane.
// The load phase has no branches: a neighbour past the degree or off the
// grid loads the record's own fields and is not selected, and the grid test
// uses no short-circuit operators, so all loads of a batch stay in flight.
template <int MAXR, bool W8, bool LIN, bool F32, bool EXACT, int DEG = 0, bool ROW = false, bool SUB = false,
          int WT0 = -1, int WT1 = -1>
__global__ __launch_bounds__(256) void stencil_kernel(const SectionArgs a) {
  const uint64_t i = (uint64_t)xcd_block(blockIdx.x, gridDim.x) * 256u + threadIdx.x;
  if (i >= (uint64_t)a.n) return;
  const uint32_t nr = EXACT ? (uint32_t)MAXR : a.n_read, nw = a.n_write;
  Acc acc[2];
  acc[0] = acc[1] = Acc{0.0f, 0.0, 0u};
  // WT0 >= 0: the fold specialised on the write types (fields of any type)
  MixFold<WT0 < 0 ? 0 : WT0, WT1 < 0 ? 3 : WT1, W8, SUB> m;
  constexpr int NB = DEG > 0 ? DEG : (MAXR >= 32 ? 1 : (MAXR <= 4 ? 8 : 32 / MAXR));
  static_assert(DEG > 0 ? DEG <= ADHA_MAX_DEGREE : ADHA_MAX_DEGREE % NB == 0,
                "batches must tile the offset tables");
  const int deg = DEG > 0 ? DEG : (int)a.degree;
  // grid coordinates of record i (a multiply and a shift per division)
  const int32_t ii = (int32_t)i;
  const uint32_t t = (uint32_t)(((uint64_t)(uint32_t)ii * a.mx) >> a.sx);
  const int32_t x = ii - (int32_t)(t * a.nx);
  int32_t z = (int32_t)(((uint64_t)t * a.my) >> a.sy);
  int32_t y = (int32_t)t - z * (int32_t)a.ny;
  if constexpr (ROW) {
    // N is a multiple of nx, hence of 64: every wave is full and in one row
    y = __builtin_amdgcn_readfirstlane(y);
    z = __builtin_amdgcn_readfirstlane(z);
  }
  uint32_t own[LIN ? MAXR : 1];
  if constexpr (LIN) {
#pragma unroll
    for (int q = 0; q < MAXR; ++q)
      own[q] = q < (int)nr ? (uint32_t)a.rd[q].base + a.rd[q].pT + (uint32_t)i * a.rd[q].TS : 0u;
  }
  for (int j0 = 0; j0 < deg; j0 += NB) {
    Words<MAXR, W8, SUB> w[NB];
    bool ok[NB];
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      // NB divides ADHA_MAX_DEGREE (or is the exact degree), so jj stays
      // inside the offset tables; entries past the degree are zero and not
      // selected
      const int jj = j0 + b;
      // a coordinate off the grid wraps to a large unsigned value
      ok[b] = (j0 + b < deg) & ((uint32_t)(x + a.off[jj][0]) < a.nx) & ((uint32_t)(y + a.off[jj][1]) < a.ny) &
              ((uint32_t)(z + a.off[jj][2]) < a.nz);
      if constexpr (LIN) {
        // the neighbour's record step (0 when it is not taken) times each
        // field's record bytes: both fit in 24 signed bits (checked at
        // launch), so one 24-bit multiply-add per field
        const int32_t d = ok[b] ? a.lin[jj] : 0;
#pragma unroll
        for (int q = 0; q < MAXR; ++q)
          if (q < (int)nr) {
            const uint32_t off = own[q] + (uint32_t)__mul24(d, (int32_t)a.rd[q].TS);
            if constexpr (SUB) w[b].load_off(q, a.buf, a.rd[q], off);
            else w[b].load_at(q, a.buf + off, a.rd[q]);
          }
      } else {
        const uint64_t rr = ok[b] ? (uint64_t)(ii + a.lin[jj]) : i;
#pragma unroll
        for (int q = 0; q < MAXR; ++q)
          if (q < (int)nr) w[b].load(q, a.buf, a.rd[q], rr);
      }
    }
    if constexpr (F32) {
#pragma unroll
      for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int q = 0; q < MAXR; ++q)
          if (q < (int)nr) {
            const float v = __uint_as_float(w[b].lo[q]);
            const float s0 = __fadd_rn(acc[0].f, v);
            acc[0].f = ok[b] ? s0 : acc[0].f;
            if (nw > 1) {
              const float s1 = __fadd_rn(__fmul_rn(acc[1].f, 0.5f), v);
              acc[1].f = ok[b] ? s1 : acc[1].f;
            }
          }
    } else if constexpr (WT0 >= 0) {
#pragma unroll
      for (int b = 0; b < NB; ++b)
#pragma unroll
        for (int q = 0; q < MAXR; ++q)
          if (q < (int)nr) m.add(a.rd[q].dt, w[b].lo[q], W8 || SUB ? w[b].hi[q] : 0u, ok[b]);
    } else {
#pragma unroll
      for (int b = 0; b < NB; ++b)
        if (ok[b]) {
#pragma unroll
          for (int q = 0; q < MAXR; ++q)
            if (q < (int)nr) {
              const uint64_t tv = w[b].term(q, a.rd[q]);
              fold(acc[0], 0, a.wr[0].dt, a.rd[q].dt, tv);
              if (nw > 1) fold(acc[1], 1, a.wr[1].dt, a.rd[q].dt, tv);
            }
        }
    }
  }
  if constexpr (F32) {
    *reinterpret_cast<uint32_t *>(a.buf + faddr(a.wr[0], i)) = __float_as_uint(acc[0].f);
    if (nw > 1) *reinterpret_cast<uint32_t *>(a.buf + faddr(a.wr[1], i)) = __float_as_uint(acc[1].f);
  } else if constexpr (WT0 >= 0) {
    m.put(a.buf, a, i);
  } else {
    store_acc(a.buf, a.wr[0], i, acc[0]);
    if (nw > 1) store_acc(a.buf, a.wr[1], i, acc[1]);
  }
}

// Gather whose read fields all sit in one interleaved group: per neighbour
// the span of the group record that holds them is fetched with VEC-byte
// vector loads (VEC divides the record size, so every load is aligned) into
// registers, and each term is picked out of those words.  One neighbour then
// costs ceil(span / VEC) wide loads instead of one load per field.
struct SpanArgs {
  uint64_t gbase;              // byte offset of the group
  uint32_t S;                  // group record bytes
  uint32_t lo;                 // first byte of the span (a multiple of VEC)
  uint32_t nvec;               // VEC-byte loads per neighbour
  uint32_t word[ADHA_MAX_READ];  // dword index of each read field inside the span
};

template <int VEC>
__device__ __forceinline__ void load_span(const uint8_t *p, uint32_t *w, int k) {
  if constexpr (VEC == 16) {
    const u32x4 v = *reinterpret_cast<const u32x4 *>(p + 16 * k);
    w[4 * k] = v.x;
    w[4 * k + 1] = v.y;
    w[4 * k + 2] = v.z;
    w[4 * k + 3] = v.w;
  } else if constexpr (VEC == 8) {
    const uint2 v = *reinterpret_cast<const uint2 *>(p + 8 * k);
    w[2 * k] = v.x;
    w[2 * k + 1] = v.y;
  } else {
    w[k] = *reinterpret_cast<const uint32_t *>(p + 4 * k);
  }
}

// w[wi] for a wave-uniform wi, as a chain of selects with constant indices
// (keeps w in registers).
template <int MAXW>
__device__ __forceinline__ uint32_t pick(const uint32_t (&w)[MAXW], uint32_t wi) {
  uint32_t r = w[0];
#pragma unroll
  for (int k = 1; k < MAXW; ++k) r = wi == (uint32_t)k ? w[k] : r;
  return r;
}

// One neighbour's span: VEC-byte loads into w (zeros when !ok).
template <int VEC, int MAXW>
__device__ __forceinline__ void span_load(const uint8_t *gb, const SpanArgs &sp, int32_t r, bool ok,
                                          uint32_t (&w)[MAXW]) {
  constexpr int WPV = VEC / 4, MAXV = MAXW / WPV;
  const uint8_t *p = gb + (uint64_t)(ok ? r : 0) * sp.S;
#pragma unroll
  for (int k = 0; k < MAXV; ++k)
    if (k < (int)sp.nvec) {
      if (ok) load_span<VEC>(p, w, k);
      else {
#pragma unroll
        for (int x = 0; x < WPV; ++x) w[WPV * k + x] = 0;
      }
    }
}

// Fold one neighbour's terms, picked out of its span in read-field order.
template <int MAXW, int MAXR>
__device__ __forceinline__ void span_fold(const SectionArgs &a, const SpanArgs &sp, const uint32_t (&w)[MAXW],
                                          Acc (&acc)[2]) {
  const uint32_t nr = a.n_read, nw = a.n_write;
  uint64_t t[MAXR];
#pragma unroll
  for (int q = 0; q < MAXR; ++q)
    if (q < (int)nr) {
      const uint32_t wi = sp.word[q];
      t[q] = pick<MAXW>(w, wi);
      if (a.rd[q].e == 8) t[q] |= (uint64_t)pick<MAXW>(w, wi + 1) << 32;
    }
#pragma unroll
  for (int q = 0; q < MAXR; ++q)
    if (q < (int)nr) {
      fold(acc[0], 0, a.wr[0].dt, a.rd[q].dt, t[q]);
      if (nw > 1) fold(acc[1], 1, a.wr[1].dt, a.rd[q].dt, t[q]);
    }
}

// One neighbour at a time (a single register array keeps the span out of
// scratch); the next neighbour's index is loaded before the current span.
// Occupancy provides the memory-level parallelism.
template <int VEC, int MAXW, int MAXR>
__global__ __launch_bounds__(256) void section_span_kernel(const SectionArgs a, const SpanArgs sp) {
  const uint64_t i = (uint64_t)blockIdx.x * 256u + threadIdx.x;
  if (i >= (uint64_t)a.n) return;
  Acc acc[2];
  acc[0] = acc[1] = Acc{0.0f, 0.0, 0u};
  const int deg = (int)a.degree;
  const Neighbours nb(a, i);
  const uint8_t *gb = a.buf + sp.gbase + sp.lo;
  int32_t cur = deg > 0 ? nb.get(a, 0) : 0;
  bool bad = false;
  for (int j = 0; j < deg; ++j) {
    const int32_t nxt = j + 1 < deg ? nb.get(a, j + 1) : 0;
    const bool ok = cur >= 0 && (int64_t)cur < a.n;
    bad |= !ok && !a.stencil;
    uint32_t w[MAXW];
    span_load<VEC, MAXW>(gb, sp, cur, ok, w);
    if (ok) span_fold<MAXW, MAXR>(a, sp, w, acc);
    cur = nxt;
  }
  if (bad) atomicOr(a.err, 1u);
  store_acc(a.buf, a.wr[0], i, acc[0]);
  if (a.n_write > 1) store_acc(a.buf, a.wr[1], i, acc[1]);
}

// The span plan of a gather, or false when its reads are not all in one
// interleaved group (or the span is wider than 16 dwords).
static bool span_plan(const SectionDesc &sec, const LayoutDesc &l, SpanArgs *sp, uint32_t *vec) {
  const uint32_t g = l.group_of[sec.rd[0]];
  for (int f : sec.rd)
    if (l.group_of[f] != g) return false;
  const Group &G = l.groups[g];
  if (G.T != 1) return false;
  uint32_t lo = ~0u, hi = 0;
  for (int f : sec.rd) {
    lo = std::min(lo, l.p[f]);
    hi = std::max(hi, l.p[f] + l.shape.ebytes[f]);
  }
  const uint32_t A = G.S % 16 == 0 ? 16 : G.S % 8 == 0 ? 8 : 4;
  const uint32_t lo_a = lo / A * A;
  const uint32_t nvec = (hi - lo_a + A - 1) / A;
  if (nvec * A / 4 > 16) return false;
  sp->gbase = G.base;
  sp->S = G.S;
  sp->lo = lo_a;
  sp->nvec = nvec;
  for (size_t q = 0; q < sec.rd.size(); ++q) sp->word[q] = (l.p[sec.rd[q]] - lo_a) / 4;
  *vec = A;
  return true;
}

template <int VEC, int MAXW>
static void launch_span_maxr(uint32_t nr, dim3 grid, const SectionArgs &a, const SpanArgs &sp, hipStream_t st) {
  if (nr <= 4) hipLaunchKernelGGL((section_span_kernel<VEC, MAXW, 4>), grid, dim3(256), 0, st, a, sp);
  else if (nr <= 8) hipLaunchKernelGGL((section_span_kernel<VEC, MAXW, 8>), grid, dim3(256), 0, st, a, sp);
  else if (nr <= 16) hipLaunchKernelGGL((section_span_kernel<VEC, MAXW, 16>), grid, dim3(256), 0, st, a, sp);
  else hipLaunchKernelGGL((section_span_kernel<VEC, MAXW, 32>), grid, dim3(256), 0, st, a, sp);
}

template <int VEC>
static void launch_span(uint32_t nr, dim3 grid, const SectionArgs &a, const SpanArgs &sp, hipStream_t st) {
  launch_span_maxr<VEC, 16>(nr, grid, a, sp, st);
}

static SField sfield(const LayoutDesc &l, int f) {
  const Group &g = l.groups[l.group_of[f]];
  SField s{};
  s.base = g.base;
  s.TS = g.T * g.S;
  s.pT = l.p[f] * g.T;
  s.logT = g.logT;
  s.e = l.shape.ebytes[f];
  s.dt = (uint32_t)l.shape.dtype[f];
  // base is a multiple of 256; the other terms of an address are multiples
  // of T*S, p*T and e
  s.al = (s.e % 4 == 0 && s.TS % 4 == 0 && s.pT % 4 == 0) ? 1u : 0u;
  return s;
}

// Kernels for sections with a field narrower than 4 bytes or a field that is
// not 4-byte aligned in the layout: the generic kernel reading every field
// through load_any.
template <int OP, int DG>
static void launch_sub_maxr(uint32_t nr, dim3 grid, const SectionArgs &a, hipStream_t st) {
  if (nr <= 8) hipLaunchKernelGGL((section_kernel<OP, DG, 8, true, true>), grid, dim3(256), 0, st, a);
  else hipLaunchKernelGGL((section_kernel<OP, DG, 32, true, true>), grid, dim3(256), 0, st, a);
}

// Stencils that are not all F32, up to 8 read fields: every field through
// load_any (any type, width and alignment) and MixFold for the write types.
// W8: some read field is 8 bytes wide (the forms without linear offsets
// always take W8).
template <int MAXR, bool LIN, bool W8, int WT0>
static void launch_stencil_mixed_w1(int wt1, dim3 grid, const SectionArgs &a, hipStream_t st) {
  switch (wt1) {
    case 0: hipLaunchKernelGGL((stencil_kernel<MAXR, W8, LIN, false, false, 0, false, true, WT0, 0>), grid, dim3(256), 0, st, a); break;
    case 1: hipLaunchKernelGGL((stencil_kernel<MAXR, W8, LIN, false, false, 0, false, true, WT0, 1>), grid, dim3(256), 0, st, a); break;
    case 2: hipLaunchKernelGGL((stencil_kernel<MAXR, W8, LIN, false, false, 0, false, true, WT0, 2>), grid, dim3(256), 0, st, a); break;
    default: hipLaunchKernelGGL((stencil_kernel<MAXR, W8, LIN, false, false, 0, false, true, WT0, 3>), grid, dim3(256), 0, st, a); break;
  }
}

template <int MAXR, bool LIN, bool W8>
static void launch_stencil_mixed(int wt0, int wt1, dim3 grid, const SectionArgs &a, hipStream_t st) {
  if (wt0 == 0) launch_stencil_mixed_w1<MAXR, LIN, W8, 0>(wt1, grid, a, st);
  else if (wt0 == 1) launch_stencil_mixed_w1<MAXR, LIN, W8, 1>(wt1, grid, a, st);
  else launch_stencil_mixed_w1<MAXR, LIN, W8, 2>(wt1, grid, a, st);
}

// The stencil kernel's linear-offset forms apply: the layout fits in 4 GiB,
// every read field sits in a group with T = 1 (its offset is base + p +
// r*S), and each neighbour's record step, its product with a field's record
// bytes and that record size fit the 24-bit multiply-add and 32-bit sums.
static bool stencil_linear(const SectionArgs &a, const LayoutDesc &l) {
  bool lin = l.nbytes <= (1ull << 32);
  int64_t max_lin = 0;
  for (uint32_t j = 0; j < a.degree; ++j) max_lin = std::max<int64_t>(max_lin, std::abs((int64_t)a.lin[j]));
  lin &= max_lin < (1 << 23);
  for (uint32_t q = 0; q < a.n_read; ++q)
    lin &= a.rd[q].logT == 0 && a.rd[q].TS < (1u << 23) && max_lin * (int64_t)a.rd[q].TS < (int64_t(1) << 31);
  return lin;
}

static void launch_sub(const SectionDesc &sec, uint32_t nr, dim3 grid, const SectionArgs &a, hipStream_t st) {
  if (sec.stencil) {
    // more than 8 read fields: the stencil kernel's generic fold, every
    // field through load_any
    hipLaunchKernelGGL((stencil_kernel<32, true, false, false, false, 0, false, true>), grid, dim3(256), 0, st, a);
    return;
  }
  switch (sec.op) {
    case ADHA_OP_GEN:
      if (sec.degree == 0) launch_sub_maxr<ADHA_OP_GEN, 0>(nr, grid, a, st);
      else if (sec.degree <= 8) launch_sub_maxr<ADHA_OP_GEN, 8>(nr, grid, a, st);
      else if (sec.degree <= 16) launch_sub_maxr<ADHA_OP_GEN, 16>(nr, grid, a, st);
      else launch_sub_maxr<ADHA_OP_GEN, 32>(nr, grid, a, st);
      break;
    case ADHA_OP_SUM: launch_sub_maxr<ADHA_OP_SUM, 0>(nr, grid, a, st); break;
    case ADHA_OP_MULADD3:
      hipLaunchKernelGGL((section_kernel<ADHA_OP_MULADD3, 0, 4, true, true>), grid, dim3(256), 0, st, a);
      break;
    default:
      hipLaunchKernelGGL((section_kernel<ADHA_OP_SUB2, 0, 4, true, true>), grid, dim3(256), 0, st, a);
      break;
  }
}

template <bool LIN, int DEG, bool ROW>
static void launch_stencil_f32_exact(uint32_t nr, dim3 grid, const SectionArgs &a, hipStream_t st) {
  if (nr == 1) hipLaunchKernelGGL((stencil_kernel<1, false, LIN, true, true, DEG, ROW>), grid, dim3(256), 0, st, a);
  else if (nr == 2) hipLaunchKernelGGL((stencil_kernel<2, false, LIN, true, true, DEG, ROW>), grid, dim3(256), 0, st, a);
  else if (nr == 3) hipLaunchKernelGGL((stencil_kernel<3, false, LIN, true, true, DEG, ROW>), grid, dim3(256), 0, st, a);
  else hipLaunchKernelGGL((stencil_kernel<4, false, LIN, true, true, DEG, ROW>), grid, dim3(256), 0, st, a);
}

template <bool W8, bool LIN, bool F32>
static void launch_stencil(uint32_t nr, dim3 grid, const SectionArgs &a, hipStream_t st) {
  if constexpr (F32 && LIN) {
    // the common small stencils: exact field count, 7 neighbours, rows of a
    // multiple of 64 records
    if (nr >= 1 && nr <= 4) {
      const bool row = a.nx % 64 == 0, d7 = a.degree == 7;
      if (row && d7) launch_stencil_f32_exact<true, 7, true>(nr, grid, a, st);
      else if (row) launch_stencil_f32_exact<true, 0, true>(nr, grid, a, st);
      else if (d7) launch_stencil_f32_exact<true, 7, false>(nr, grid, a, st);
      else launch_stencil_f32_exact<true, 0, false>(nr, grid, a, st);
      return;
    }
  }
  if constexpr (F32) {
    // exact field counts for the small stencils (the common case)
    if (nr == 1) {
      hipLaunchKernelGGL((stencil_kernel<1, W8, LIN, F32, true>), grid, dim3(256), 0, st, a);
      return;
    }
    if (nr == 2) {
      hipLaunchKernelGGL((stencil_kernel<2, W8, LIN, F32, true>), grid, dim3(256), 0, st, a);
      return;
    }
    if (nr == 3) {
      hipLaunchKernelGGL((stencil_kernel<3, W8, LIN, F32, true>), grid, dim3(256), 0, st, a);
      return;
    }
    if (nr == 4) {
      hipLaunchKernelGGL((stencil_kernel<4, W8, LIN, F32, true>), grid, dim3(256), 0, st, a);
      return;
    }
  }
  if (nr <= 4) hipLaunchKernelGGL((stencil_kernel<4, W8, LIN, F32, false>), grid, dim3(256), 0, st, a);
  else if (nr <= 8) hipLaunchKernelGGL((stencil_kernel<8, W8, LIN, F32, false>), grid, dim3(256), 0, st, a);
  else if (nr <= 16) hipLaunchKernelGGL((stencil_kernel<16, W8, LIN, F32, false>), grid, dim3(256), 0, st, a);
  else hipLaunchKernelGGL((stencil_kernel<32, W8, LIN, F32, false>), grid, dim3(256), 0, st, a);
}

template <int OP, int DG, bool W8>
static void launch_maxr_w(uint32_t nr, dim3 grid, const SectionArgs &a, hipStream_t st) {
  if (nr <= 4) hipLaunchKernelGGL((section_kernel<OP, DG, 4, W8>), grid, dim3(256), 0, st, a);
  else if (nr <= 8) hipLaunchKernelGGL((section_kernel<OP, DG, 8, W8>), grid, dim3(256), 0, st, a);
  else if (nr <= 16) hipLaunchKernelGGL((section_kernel<OP, DG, 16, W8>), grid, dim3(256), 0, st, a);
  else hipLaunchKernelGGL((section_kernel<OP, DG, 32, W8>), grid, dim3(256), 0, st, a);
}

template <bool LIN>
static void launch_direct_f32(uint32_t nr, dim3 grid, const SectionArgs &a, hipStream_t st) {
  // up to 4 reads: 4 records per thread
  const dim3 grid4((uint32_t)(((uint64_t)a.n + 1023) / 1024));
  if (nr <= 4) hipLaunchKernelGGL((direct_f32_kernel<4, LIN, 4>), grid4, dim3(256), 0, st, a);
  else if (nr <= 8) hipLaunchKernelGGL((direct_f32_kernel<8, LIN, 1>), grid, dim3(256), 0, st, a);
  else if (nr <= 16) hipLaunchKernelGGL((direct_f32_kernel<16, LIN, 1>), grid, dim3(256), 0, st, a);
  else hipLaunchKernelGGL((direct_f32_kernel<32, LIN, 1>), grid, dim3(256), 0, st, a);
}

template <int OP, int DG>
static void launch_maxr(uint32_t nr, dim3 grid, const SectionArgs &a, hipStream_t st) {
  bool w8 = false;
  for (uint32_t q = 0; q < nr; ++q) w8 |= a.rd[q].e == 8;
  if (w8) launch_maxr_w<OP, DG, true>(nr, grid, a, st);
  else launch_maxr_w<OP, DG, false>(nr, grid, a, st);
}

// ------------------------------------------------------------ reductions
// A reduction adds the read fields of every record into row `key` of a small
// table; the last column counts records.  Integer fields are summed in int64
// (two's complement), which is exact in any order.  Floating-point fields are
// summed in double with compensation, in an order fixed by N and the grid:
//  * each thread walks its records in a fixed grid-stride sequence and keeps
//    per cell a pair (s, c): s the rounded running sum, c the sum of the
//    exact rounding errors of s (Knuth's TwoSum; Ogita, Rump and Oishi's
//    Sum2), so s + c carries about twice the precision of a double;
//  * pairs are then combined pairwise with TwoSum on both parts and
//    renormalised (double-double addition) in fixed trees: the 64 lanes of a
//    wave by a butterfly, the waves of a workgroup in order, and in pass 2
//    the workgroups of a cell (strided per thread, then a tree in LDS);
//  * the table gets the double nearest the final pair.
// No floating-point atomics are used anywhere, so two runs on one device give
// the same bits.
// Pass 1 has two forms:
//  * at most 8 keys: every thread keeps its pairs for a slice of the table's
//    columns in registers; gridDim.y runs over the slices;
//  * more keys: one wave per workgroup with its own table in LDS.  Lanes of
//    one wave that hit the same key add in lane order: a lane's rank among
//    the lanes with its key is found with ballots, and the wave adds in
//    rounds of rank 0, 1, ..., so no two lanes of a round touch one row.
// Either way pass 1 writes one partial table of pairs per workgroup.
struct ReduceArgs {
  const uint8_t *buf;
  uint32_t *err;
  uint64_t *partials;  // [cells][gridDim.x][2]: a pair (s, c) of doubles, or an int64 and a zero word
  int64_t n;
  uint32_t n_read, n_keys, cells, has_key;
  uint32_t fp_mask;    // bit q: read field q is floating point
  uint32_t plain;      // 1: plain double sums in the same order (no compensation)
  SField rd[ADHA_MAX_READ];
  SField key;
};

// s + e = a + b exactly with s = fl(a + b), for any doubles a, b (no
// ordering of the operands needed; Knuth's TwoSum).
__device__ __forceinline__ void two_sum(double a, double b, double &s, double &e) {
  const double t = __dadd_rn(a, b);
  const double bb = __dsub_rn(t, a);
  e = __dadd_rn(__dsub_rn(a, __dsub_rn(t, bb)), __dsub_rn(b, bb));
  s = t;
}

// One value into a compensated pair (s, c).  PLAIN: s += v only.
template <bool PLAIN>
__device__ __forceinline__ void comp_add(double &s, double &c, double v) {
  if constexpr (PLAIN) {
    s = __dadd_rn(s, v);
  } else {
    double e;
    two_sum(s, v, s, e);
    c = __dadd_rn(c, e);
  }
}

// (a1 + a2) + (b1 + b2) as a pair (hi, lo) with hi = fl(hi + lo).  Every
// step but two is exact; the two roundings are of quantities of the order of
// the low parts, so the pair keeps about 106 bits of the exact sum.
__device__ __forceinline__ void pair_add(double a1, double a2, double b1, double b2, double &hi, double &lo) {
  double s, e, t, f, s2, e3;
  two_sum(a1, b1, s, e);
  two_sum(a2, b2, t, f);
  two_sum(s, __dadd_rn(e, t), s2, e3);
  two_sum(s2, __dadd_rn(e3, f), hi, lo);
}

__device__ __forceinline__ double bits_f64(uint64_t b) { return __longlong_as_double((long long)b); }
__device__ __forceinline__ uint64_t f64_bits(double d) { return (uint64_t)__double_as_longlong(d); }

__device__ __forceinline__ void wave_pair_sum(double &hi, double &lo) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) {
    const double oh = __shfl_xor(hi, m, 64), ol = __shfl_xor(lo, m, 64);
    pair_add(hi, lo, oh, ol, hi, lo);
  }
}

__device__ __forceinline__ uint64_t wave_sum_u64(uint64_t v) {
#pragma unroll
  for (int m = 32; m >= 1; m >>= 1) v += (uint64_t)__shfl_xor((long long)v, m, 64);
  return v;
}

// An integer column's term as int64 bits (I32 sign-extended, U32 zero-extended).
__device__ __forceinline__ uint64_t int_col(uint32_t dt, uint64_t t) { return (uint64_t)int_value(dt, t); }

// End of a register-form workgroup: per cell of the slice, the wave sums
// (lane 0 of each wave into LDS), then the 4 waves in order, into the
// workgroup's partial.  fp(c) tells a floating-point column slot; hi/lo hold
// a pair (or hi the int64 bits) per (key, slot).
template <int KR, int CR, class IsFp>
__device__ __forceinline__ void reduce_reg_finish(const ReduceArgs &a, uint64_t (&hi)[KR][CR], double (&lo)[KR][CR],
                                                  uint32_t c0, uint32_t nc, IsFp fp) {
  __shared__ uint64_t wsum[4][KR * CR][2];
  const uint32_t wave = threadIdx.x >> 6, lane = threadIdx.x & 63u;
#pragma unroll
  for (int c = 0; c < CR; ++c) {
#pragma unroll
    for (int kk = 0; kk < KR; ++kk) {
      if (fp(c)) {
        double h = bits_f64(hi[kk][c]), l = lo[kk][c];
        wave_pair_sum(h, l);
        if (lane == 0) {
          wsum[wave][kk * CR + c][0] = f64_bits(h);
          wsum[wave][kk * CR + c][1] = f64_bits(l);
        }
      } else {
        const uint64_t u = wave_sum_u64(hi[kk][c]);
        if (lane == 0) {
          wsum[wave][kk * CR + c][0] = u;
          wsum[wave][kk * CR + c][1] = 0;
        }
      }
    }
  }
  __syncthreads();
  const uint32_t t = threadIdx.x;
  if (t < (uint32_t)(KR * CR)) {
    const uint32_t kk = t / CR, c = t % CR, col = c0 + c;
    if (kk < a.n_keys && c < nc) {
      const uint32_t cols = a.n_read + 1;
      uint64_t o0, o1;
      if (fp(c)) {
        double h = bits_f64(wsum[0][t][0]), l = bits_f64(wsum[0][t][1]);
        for (int w = 1; w < 4; ++w) pair_add(h, l, bits_f64(wsum[w][t][0]), bits_f64(wsum[w][t][1]), h, l);
        o0 = f64_bits(h);
        o1 = f64_bits(l);
      } else {
        o0 = wsum[0][t][0] + wsum[1][t][0] + wsum[2][t][0] + wsum[3][t][0];
        o1 = 0;
      }
      const uint64_t at = ((uint64_t)(kk * cols + col) * gridDim.x + blockIdx.x) * 2;
      a.partials[at] = o0;
      a.partials[at + 1] = o1;
    }
  }
}

// Few keys: pairs in registers.  KR >= n_keys rows, CR columns per slice.
template <int KR, int CR, bool W8, bool PLAIN>
__global__ __launch_bounds__(256) void reduce_reg_kernel(const ReduceArgs a) {
  const uint32_t nr = a.n_read, cols = nr + 1;
  const uint32_t c0 = blockIdx.y * CR;
  const uint32_t nc = min((uint32_t)CR, cols - c0);
  uint64_t hi[KR][CR];  // fp: bits of s; integer and count columns: int64
  double lo[KR][CR];
#pragma unroll
  for (int kk = 0; kk < KR; ++kk)
#pragma unroll
    for (int c = 0; c < CR; ++c) {
      hi[kk][c] = 0;
      lo[kk][c] = 0.0;
    }
  bool bad = false;
  const uint64_t stride = (uint64_t)gridDim.x * 256u;
  for (uint64_t i = (uint64_t)blockIdx.x * 256u + threadIdx.x; i < (uint64_t)a.n; i += stride) {
    int32_t k = 0;
    if (a.has_key) k = (int32_t)load_word(a.buf, a.key, i);
    const bool ok = k >= 0 && (uint32_t)k < a.n_keys;
    bad |= !ok;
    // every slot loads, with no branch around the loads (a slot past the
    // reads uses the last descriptor, zeroed unless all 32 are reads, and
    // its value is dropped), so they are in flight together
    Words<CR, W8> w;
#pragma unroll
    for (int c = 0; c < CR; ++c) w.load(c, a.buf, a.rd[c0 + c < nr ? c0 + c : ADHA_MAX_READ - 1], i);
    uint64_t v[CR];
#pragma unroll
    for (int c = 0; c < CR; ++c) v[c] = c0 + c < nr ? w.term(c, a.rd[c0 + c]) : 1;
#pragma unroll
    for (int c = 0; c < CR; ++c) {
      if ((uint32_t)c >= nc) continue;
      const uint32_t col = c0 + c;
      if (col < nr && (a.fp_mask >> col & 1u)) {
        const double d = to_f64(a.rd[col].dt, v[c]);
#pragma unroll
        for (int kk = 0; kk < KR; ++kk) {
          // adding +0.0 leaves a pair unchanged bit for bit
          double s = bits_f64(hi[kk][c]);
          comp_add<PLAIN>(s, lo[kk][c], (ok && k == kk) ? d : 0.0);
          hi[kk][c] = f64_bits(s);
        }
      } else {
        const uint64_t u = col < nr ? int_col(a.rd[col].dt, v[c]) : v[c];
#pragma unroll
        for (int kk = 0; kk < KR; ++kk) hi[kk][c] = (ok && k == kk) ? hi[kk][c] + u : hi[kk][c];
      }
    }
  }
  reduce_reg_finish<KR, CR>(a, hi, lo, c0, nc,
                            [&](int c) { return c0 + c < nr && (a.fp_mask >> (c0 + c) & 1u); });
  if (bad) atomicOr(a.err, 1u);
}

// Few keys, every read field F32: the same pairs with no branch per column.
// A column slot past the reads folds +0.0, and the record counts live in
// their own per-key registers, written by the slice that holds the count
// column.  LIN: the read fields and the key sit in groups with T = 1 and the
// layout fits in 4 GiB, so offsets are base + p + r*S in 32 bits.
template <bool LIN>
__device__ __forceinline__ uint32_t reduce_word(const ReduceArgs &a, const SField &F, uint64_t i) {
  if constexpr (LIN) return *reinterpret_cast<const uint32_t *>(a.buf + ((uint32_t)F.base + F.pT + (uint32_t)i * F.TS));
  return load_word(a.buf, F, i);
}

template <int KR, int CR, bool LIN, bool PLAIN>
__global__ __launch_bounds__(256) void reduce_reg_f32_kernel(const ReduceArgs a) {
  const uint32_t nr = a.n_read, cols = nr + 1;
  const uint32_t c0 = blockIdx.y * CR;
  const uint32_t nc = min((uint32_t)CR, cols - c0);
  double s[KR][CR], lo[KR][CR];
  uint32_t cnt[KR];
#pragma unroll
  for (int kk = 0; kk < KR; ++kk) {
    cnt[kk] = 0;
#pragma unroll
    for (int c = 0; c < CR; ++c) s[kk][c] = lo[kk][c] = 0.0;
  }
  bool bad = false;
  const uint64_t stride = (uint64_t)gridDim.x * 256u;
  for (uint64_t i = (uint64_t)blockIdx.x * 256u + threadIdx.x; i < (uint64_t)a.n; i += stride) {
    int32_t k = 0;
    if (a.has_key) k = (int32_t)reduce_word<LIN>(a, a.key, i);
    const bool ok = k >= 0 && (uint32_t)k < a.n_keys;
    bad |= !ok;
    uint32_t w[CR];
#pragma unroll
    for (int c = 0; c < CR; ++c) w[c] = reduce_word<LIN>(a, a.rd[c0 + c < nr ? c0 + c : ADHA_MAX_READ - 1], i);
#pragma unroll
    for (int c = 0; c < CR; ++c) {
      const double d = c0 + c < nr ? (double)__uint_as_float(w[c]) : 0.0;
#pragma unroll
      for (int kk = 0; kk < KR; ++kk) comp_add<PLAIN>(s[kk][c], lo[kk][c], (ok && k == kk) ? d : 0.0);
    }
#pragma unroll
    for (int kk = 0; kk < KR; ++kk) cnt[kk] += (ok && k == kk) ? 1u : 0u;
  }
  // the count column takes the slot of the first column past the reads
  uint64_t hi[KR][CR];
#pragma unroll
  for (int kk = 0; kk < KR; ++kk)
#pragma unroll
    for (int c = 0; c < CR; ++c) hi[kk][c] = c0 + c == nr ? (uint64_t)cnt[kk] : f64_bits(s[kk][c]);
  reduce_reg_finish<KR, CR>(a, hi, lo, c0, nc, [&](int c) { return c0 + c < nr; });
  if (bad) atomicOr(a.err, 1u);
}

// 3 to 8 keys, every read field F32: the slot form.  Each thread keeps its
// pairs for a slice of CR columns in LDS, slot[(key * CR + c) * 128 + t], so
// a value costs one TwoSum at its record's key (the register form spends one
// per key, selecting which to keep).  128 threads; a thread walks its
// records U at a time (all loads first, then the adds in record order).
constexpr uint32_t kSlotThreads = 128;

// The slot form's end: the pairs of the C = K * CR cells (cell x = key * CR
// + column slot) reduced over the workgroup's threads in a fixed tree, then
// written as the workgroup's partial.  Recursive halving first: at mask m
// (1, 2, .., P/2; P the power of two >= C) thread t keeps half of its cell
// range -- the upper half when t & m -- and adds thread t ^ m's pair for
// each cell of it, the lower thread's pair first; after it thread t holds
// one cell summed over the P threads that share its high bits.  Those
// groups are then added pairwise in order of t, and thread t < P writes
// cell x(t).  A barrier separates the levels.  Pairs are added with
// pair_add, count cells as integers.
template <int CR>
__device__ __forceinline__ void reduce_slot_finish(const ReduceArgs &a, double2 *slot, uint32_t K, uint32_t c0,
                                                   uint32_t nc) {
  const uint32_t t = threadIdx.x, nr = a.n_read, cols = nr + 1;
  const uint32_t C = K * CR;
  uint32_t P = 1;
  while (P < C) P <<= 1;
  auto is_count = [&](uint32_t x) { return c0 + x % CR == nr; };
  auto add = [&](uint32_t x, double2 lo_t, double2 hi_t) {
    double2 r;
    if (is_count(x)) {
      r.x = bits_f64(f64_bits(lo_t.x) + f64_bits(hi_t.x));
      r.y = 0.0;
    } else {
      pair_add(lo_t.x, lo_t.y, hi_t.x, hi_t.y, r.x, r.y);
    }
    return r;
  };
  uint32_t first = 0, span = P;
  for (uint32_t m = 1; m < P; m <<= 1) {
    span >>= 1;
    const bool upper = (t & m) != 0;
    if (upper) first += span;
    __syncthreads();
    for (uint32_t x = first; x < first + span; ++x) {
      if (x >= C) break;
      const double2 mine = slot[x * kSlotThreads + t], other = slot[x * kSlotThreads + (t ^ m)];
      slot[x * kSlotThreads + t] = upper ? add(x, other, mine) : add(x, mine, other);
    }
  }
  // thread t now holds cell `first` (if below C), summed over its P-group
  for (uint32_t m = P; m < kSlotThreads; m <<= 1) {
    __syncthreads();
    if ((t & (2 * m - 1)) < P && first < C) {
      // t is the lowest thread of its 2m-block holding this cell
      slot[first * kSlotThreads + t] = add(first, slot[first * kSlotThreads + t], slot[first * kSlotThreads + t + m]);
    }
  }
  __syncthreads();
  if (t < P && first < C) {
    const uint32_t kk = first / CR, c = first % CR, col = c0 + c;
    if (c < nc && kk < a.n_keys) {
      const double2 v = slot[first * kSlotThreads + t];
      const uint64_t at = ((uint64_t)(kk * cols + col) * gridDim.x + blockIdx.x) * 2;
      a.partials[at] = f64_bits(v.x);
      a.partials[at + 1] = is_count(first) ? 0 : f64_bits(v.y);
    }
  }
}

template <int CR, bool LIN, bool PLAIN>
__global__ __launch_bounds__(kSlotThreads) void reduce_slot_f32_kernel(const ReduceArgs a) {
  extern __shared__ double2 slot[];  // [K * CR][kSlotThreads]
  constexpr int U = 8;
  const uint32_t nr = a.n_read, cols = nr + 1, K = a.n_keys, t = threadIdx.x;
  const uint32_t c0 = blockIdx.y * CR;
  const uint32_t nc = min((uint32_t)CR, cols - c0);
  for (uint32_t x = 0; x < K * CR; ++x) slot[x * kSlotThreads + t] = make_double2(0.0, 0.0);
  bool bad = false;
  const uint64_t stride = (uint64_t)gridDim.x * kSlotThreads;
  for (uint64_t i0 = (uint64_t)blockIdx.x * kSlotThreads + t; i0 < (uint64_t)a.n; i0 += U * stride) {
    // U records: i0, i0 + stride, ...: keys and words loaded first
    int32_t k[U];
    uint32_t w[U][CR];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const uint64_t i = i0 + u * stride;
      const bool live = i < (uint64_t)a.n;
      const uint64_t r = live ? i : 0;  // past N: record 0, dropped below
      k[u] = a.has_key ? (int32_t)reduce_word<LIN>(a, a.key, r) : 0;
      if (!live) k[u] = -1;
#pragma unroll
      for (int c = 0; c < CR; ++c) w[u][c] = reduce_word<LIN>(a, a.rd[c0 + c < nr ? c0 + c : ADHA_MAX_READ - 1], r);
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const bool live = i0 + u * stride < (uint64_t)a.n;
      const bool ok = k[u] >= 0 && (uint32_t)k[u] < K;
      bad |= live && !ok;
      if (!ok) continue;
      double2 *row = slot + (uint32_t)k[u] * CR * kSlotThreads + t;
#pragma unroll
      for (int c = 0; c < CR; ++c) {
        if ((uint32_t)c >= nc) continue;
        double2 q = row[c * kSlotThreads];
        if (c0 + c < nr) comp_add<PLAIN>(q.x, q.y, (double)__uint_as_float(w[u][c]));
        else q.x = bits_f64(f64_bits(q.x) + 1);  // the count column: an int64 in the first word
        row[c * kSlotThreads] = q;
      }
    }
  }
  reduce_slot_finish<CR>(a, slot, K, c0, nc);
  if (bad) atomicOr(a.err, 1u);
}

// More keys: one wave per workgroup, with its own table of pairs in LDS.
template <int MAXR, bool W8, bool PLAIN>
__global__ __launch_bounds__(64) void reduce_lds_kernel(const ReduceArgs a) {
  extern __shared__ uint64_t tab[];  // [cells][2]
  const uint32_t nr = a.n_read, cols = nr + 1, cells = a.cells;
  const uint32_t lane = threadIdx.x;
  for (uint32_t c = lane; c < 2 * cells; c += 64) tab[c] = 0;
  __syncthreads();
  bool bad = false;
  const uint64_t stride = (uint64_t)gridDim.x * 64u;
  for (uint64_t i0 = (uint64_t)blockIdx.x * 64u; i0 < (uint64_t)a.n; i0 += stride) {
    const uint64_t i = i0 + lane;
    const bool live = i < (uint64_t)a.n;
    int32_t k = 0;
    if (a.has_key && live) k = (int32_t)load_word(a.buf, a.key, i);
    const bool ok = live && k >= 0 && (uint32_t)k < a.n_keys;
    bad |= live && !ok;
    Words<MAXR, W8> w;
    const uint64_t rr = live ? i : 0;  // lanes past N load record 0, unused
#pragma unroll
    for (int q = 0; q < MAXR; ++q)
      if (q < (int)nr) w.load(q, a.buf, a.rd[q], rr);
    // the terms as doubles (floating-point fields) or int64 bits (I32)
    uint64_t v[MAXR];
#pragma unroll
    for (int q = 0; q < MAXR; ++q) {
      const uint64_t t = q < (int)nr ? w.term(q, a.rd[q]) : 0;
      v[q] = (a.fp_mask >> q & 1u) ? f64_bits(to_f64(a.rd[q].dt, t)) : int_col(a.rd[q].dt, t);
    }
    // rank of each lane among the lanes with its key, in lane order, and the
    // number of rounds (the largest count of one key)
    uint64_t pending = __ballot(ok);
    uint32_t rank = 0, rounds = 0;
    const uint64_t below = (1ull << lane) - 1ull;
    while (pending) {
      const int leader = __ffsll((unsigned long long)pending) - 1;
      const int32_t lk = __shfl(k, leader, 64);
      const bool same = ok && k == lk;
      const uint64_t m = __ballot(same);
      if (same) rank = (uint32_t)__popcll(m & below);
      rounds = max(rounds, (uint32_t)__popcll(m));
      pending &= ~m;
    }
    for (uint32_t r = 0; r < rounds; ++r) {
      if (ok && rank == r) {
        uint64_t *row = tab + (uint64_t)(uint32_t)k * cols * 2;
#pragma unroll
        for (int q = 0; q < MAXR; ++q)
          if (q < (int)nr) {
            if (a.fp_mask >> q & 1u) {
              double sv = bits_f64(row[2 * q]), cv = bits_f64(row[2 * q + 1]);
              comp_add<PLAIN>(sv, cv, bits_f64(v[q]));
              // a cell's chain is every record of the workgroup with that
              // key, so the pair is renormalised after each value: its error
              // then grows with the chain's length, not with its square
              if constexpr (!PLAIN) two_sum(sv, cv, sv, cv);
              row[2 * q] = f64_bits(sv);
              row[2 * q + 1] = f64_bits(cv);
            } else {
              row[2 * q] += v[q];
            }
          }
        row[2 * nr] += 1;
      }
      __syncthreads();
    }
  }
  __syncthreads();
  for (uint32_t c = lane; c < cells; c += 64) {
    const uint64_t at = ((uint64_t)c * gridDim.x + blockIdx.x) * 2;
    a.partials[at] = tab[2 * c];
    a.partials[at + 1] = tab[2 * c + 1];
  }
  if (bad) atomicOr(a.err, 1u);
}

// Pass 2: one workgroup per cell adds the workgroups' partials, each thread
// striding over them in order, then a tree in LDS.
template <bool PLAIN>
__global__ __launch_bounds__(256) void reduce_final_kernel(const uint64_t *partials, uint32_t groups, uint32_t cols,
                                                           uint32_t fp_mask, uint64_t *out) {
  __shared__ double sh[256], sl[256];
  __shared__ uint64_t su[256];
  const uint32_t c = blockIdx.x, q = c % cols;
  const bool fp = q + 1 < cols && (fp_mask >> q & 1u);
  const uint64_t *p = partials + (uint64_t)c * groups * 2;
  double h = 0.0, l = 0.0;
  uint64_t u = 0;
  for (uint32_t g = threadIdx.x; g < groups; g += 256) {
    if (fp) {
      if constexpr (PLAIN) h = __dadd_rn(h, bits_f64(p[2 * g]));
      else pair_add(h, l, bits_f64(p[2 * g]), bits_f64(p[2 * g + 1]), h, l);
    } else {
      u += p[2 * g];
    }
  }
  sh[threadIdx.x] = h;
  sl[threadIdx.x] = l;
  su[threadIdx.x] = u;
  __syncthreads();
  for (uint32_t w = 128; w >= 1; w >>= 1) {
    if (threadIdx.x < w) {
      const uint32_t t = threadIdx.x;
      if constexpr (PLAIN) {
        sh[t] = __dadd_rn(sh[t], sh[t + w]);
      } else {
        double hh, ll;
        pair_add(sh[t], sl[t], sh[t + w], sl[t + w], hh, ll);
        sh[t] = hh;
        sl[t] = ll;
      }
      su[threadIdx.x] += su[threadIdx.x + w];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) out[c] = fp ? f64_bits(sh[0]) : su[0];
}

template <bool W8, bool PLAIN>
static void reduce_dispatch(uint32_t KR, uint32_t nr, dim3 grid, size_t lds, hipStream_t stream, const ReduceArgs &a) {
  switch (KR) {
    case 1: hipLaunchKernelGGL((reduce_reg_kernel<1, 17, W8, PLAIN>), grid, dim3(256), 0, stream, a); return;
    case 2: hipLaunchKernelGGL((reduce_reg_kernel<2, 9, W8, PLAIN>), grid, dim3(256), 0, stream, a); return;
    case 3: hipLaunchKernelGGL((reduce_reg_kernel<3, 6, W8, PLAIN>), grid, dim3(256), 0, stream, a); return;
    case 4: hipLaunchKernelGGL((reduce_reg_kernel<4, 5, W8, PLAIN>), grid, dim3(256), 0, stream, a); return;
    case 5: hipLaunchKernelGGL((reduce_reg_kernel<5, 4, W8, PLAIN>), grid, dim3(256), 0, stream, a); return;
    case 6: hipLaunchKernelGGL((reduce_reg_kernel<6, 3, W8, PLAIN>), grid, dim3(256), 0, stream, a); return;
    case 7: hipLaunchKernelGGL((reduce_reg_kernel<7, 3, W8, PLAIN>), grid, dim3(256), 0, stream, a); return;
    case 8: hipLaunchKernelGGL((reduce_reg_kernel<8, 3, W8, PLAIN>), grid, dim3(256), 0, stream, a); return;
    default: break;
  }
  if (nr <= 4) hipLaunchKernelGGL((reduce_lds_kernel<4, W8, PLAIN>), grid, dim3(64), lds, stream, a);
  else if (nr <= 8) hipLaunchKernelGGL((reduce_lds_kernel<8, W8, PLAIN>), grid, dim3(64), lds, stream, a);
  else if (nr <= 16) hipLaunchKernelGGL((reduce_lds_kernel<16, W8, PLAIN>), grid, dim3(64), lds, stream, a);
  else hipLaunchKernelGGL((reduce_lds_kernel<32, W8, PLAIN>), grid, dim3(64), lds, stream, a);
}

template <bool LIN, bool PLAIN>
static void reduce_f32_dispatch(uint32_t KR, dim3 grid, hipStream_t stream, const ReduceArgs &a) {
  switch (KR) {
    case 1: hipLaunchKernelGGL((reduce_reg_f32_kernel<1, 17, LIN, PLAIN>), grid, dim3(256), 0, stream, a); break;
    case 2: hipLaunchKernelGGL((reduce_reg_f32_kernel<2, 9, LIN, PLAIN>), grid, dim3(256), 0, stream, a); break;
    case 3: hipLaunchKernelGGL((reduce_reg_f32_kernel<3, 6, LIN, PLAIN>), grid, dim3(256), 0, stream, a); break;
    case 4: hipLaunchKernelGGL((reduce_reg_f32_kernel<4, 5, LIN, PLAIN>), grid, dim3(256), 0, stream, a); break;
    case 5: hipLaunchKernelGGL((reduce_reg_f32_kernel<5, 4, LIN, PLAIN>), grid, dim3(256), 0, stream, a); break;
    case 6: hipLaunchKernelGGL((reduce_reg_f32_kernel<6, 3, LIN, PLAIN>), grid, dim3(256), 0, stream, a); break;
    case 7: hipLaunchKernelGGL((reduce_reg_f32_kernel<7, 3, LIN, PLAIN>), grid, dim3(256), 0, stream, a); break;
    default: hipLaunchKernelGGL((reduce_reg_f32_kernel<8, 3, LIN, PLAIN>), grid, dim3(256), 0, stream, a); break;
  }
}

// Register slice widths per key count (pairs per thread: keys x columns).
static const uint32_t kRedCols[9] = {0, 17, 9, 6, 5, 4, 3, 3, 3};
// Slot form slice widths per key count (3..8): at most 24 KB of LDS per
// workgroup, so a CU holds 6 or more of them (occupancy gains more than the
// wider slices' fewer key reads: 5 keys, 32 F32 columns, 2^23 records run
// 344 us at 2 columns per slice, 374 us at 3, 405 us at 4).
static const uint32_t kSlotCols[9] = {0, 0, 0, 3, 2, 2, 2, 2, 2};

template <bool LIN, bool PLAIN>
static void reduce_slot_dispatch(uint32_t CR, dim3 grid, size_t lds, hipStream_t stream, const ReduceArgs &a) {
  if (CR == 2) hipLaunchKernelGGL((reduce_slot_f32_kernel<2, LIN, PLAIN>), grid, dim3(kSlotThreads), lds, stream, a);
  else hipLaunchKernelGGL((reduce_slot_f32_kernel<3, LIN, PLAIN>), grid, dim3(kSlotThreads), lds, stream, a);
}

ReducePlan reduce_plan(const Ctx *ctx, const SectionDesc &sec, int64_t n) {
  ReducePlan p;
  const uint32_t cells = sec.reduce_cells(), cols = (uint32_t)sec.rd.size() + 1;
  bool f32 = true;
  for (int f : sec.rd) f32 &= sec.shape.dtype[f] == ADHA_F32;
  if (f32 && sec.n_keys >= 3 && sec.n_keys <= 8) {
    // slot form: chains of at most 64 records per thread where the partial
    // tables allow, and at least the workgroups the CUs hold at once
    p.slot_cols = kSlotCols[sec.n_keys];
    p.slices = (cols + p.slot_cols - 1) / p.slot_cols;
    p.lds = (size_t)sec.n_keys * p.slot_cols * kSlotThreads * 16;
    const uint64_t want = std::max<uint64_t>(1, ((uint64_t)n + kSlotThreads - 1) / kSlotThreads);
    const uint64_t per_cu = std::max<uint64_t>(1, 163840 / p.lds);
    const uint64_t budget = std::max<uint64_t>(1, (uint64_t)std::max(1, ctx->cu_count) * per_cu / p.slices);
    const uint64_t short_chains = ((uint64_t)n + kSlotThreads * 64 - 1) / (kSlotThreads * 64);
    const uint64_t cap = std::max<uint64_t>(1, kReducePartialPairs / cells);
    p.groups = (uint32_t)std::min<uint64_t>(std::min<uint64_t>(want, std::max(budget, short_chains)), cap);
    p.partial_bytes = (uint64_t)p.groups * cells * 16;
    return p;
  }
  p.keys_in_regs = sec.n_keys <= 8 ? sec.n_keys : 0;
  p.slices = p.keys_in_regs ? (cols + kRedCols[p.keys_in_regs] - 1) / kRedCols[p.keys_in_regs] : 1;
  const uint64_t per_wg = p.keys_in_regs ? 256 : 64;
  const uint64_t want = std::max<uint64_t>(1, ((uint64_t)n + per_wg - 1) / per_wg);
  uint64_t budget;
  if (p.keys_in_regs) {
    budget = (uint64_t)std::max(1, ctx->cu_count) * ctx->reduce_wg_per_cu / p.slices;
  } else {
    // one-wave workgroups, as many per CU as their LDS tables allow (at most 16)
    const uint64_t per_cu = std::min<uint64_t>(16, std::max<uint64_t>(1, 163840 / ((uint64_t)cells * 16)));
    budget = (uint64_t)std::max(1, ctx->cu_count) * per_cu;
  }
  // register form: enough workgroups that a thread's chain (records per
  // thread) stays within 32 where the partial tables allow it
  const uint64_t short_chains = p.keys_in_regs ? ((uint64_t)n + 256 * 32 - 1) / (256 * 32) : 1;
  const uint64_t cap = std::max<uint64_t>(1, kReducePartialPairs / cells);
  p.groups = (uint32_t)std::min<uint64_t>(std::min<uint64_t>(want, std::max<uint64_t>({1, budget, short_chains})), cap);
  p.lds = p.keys_in_regs ? 0 : (size_t)cells * 16;
  p.partial_bytes = (uint64_t)p.groups * cells * 16;
  return p;
}

adha_status reduce_launch(Ctx *ctx, const SectionDesc &sec, const LayoutDesc &l, const void *buf, void *out,
                          uint64_t *partials, uint64_t partial_cap, hipStream_t stream) {
  const int64_t n = l.shape.n;
  ReduceArgs a{};
  a.buf = (const uint8_t *)buf;
  a.err = ctx->err_flag;
  a.n = n;
  a.n_read = (uint32_t)sec.rd.size();
  a.n_keys = sec.n_keys;
  a.cells = sec.reduce_cells();
  a.has_key = sec.key >= 0;
  a.plain = ctx->reduce_plain ? 1u : 0u;
  for (size_t q = 0; q < sec.rd.size(); ++q) {
    a.rd[q] = sfield(l, sec.rd[q]);
    const int32_t dt = l.shape.dtype[sec.rd[q]];
    if (dt == ADHA_F32 || dt == ADHA_F64) a.fp_mask |= 1u << q;
    if (!a.rd[q].al)
      return fail(ADHA_ERR_UNSUPPORTED, "reduction field %d is not 4-byte aligned in this layout", sec.rd[q]);
  }
  if (sec.key >= 0) {
    a.key = sfield(l, sec.key);
    if (!a.key.al) return fail(ADHA_ERR_UNSUPPORTED, "the reduction's key is not 4-byte aligned in this layout");
  }
  const ReducePlan p = reduce_plan(ctx, sec, n);
  if (p.partial_bytes > partial_cap)
    return fail(ADHA_ERR_INVALID, "reduction partials need %llu bytes, the scratch holds %llu",
                (unsigned long long)p.partial_bytes, (unsigned long long)partial_cap);
  a.partials = partials;
  const uint32_t nr = a.n_read, cols = nr + 1, KR = p.keys_in_regs;
  const dim3 grid(p.groups, p.slices);
  bool w8 = false, f32 = true;
  for (int f : sec.rd) {
    w8 |= l.shape.ebytes[f] == 8;
    f32 &= l.shape.dtype[f] == ADHA_F32;
  }
  const bool plain = a.plain != 0;
  if (p.slot_cols) {
    bool lin = l.nbytes <= (1ull << 32) && (sec.key < 0 || a.key.logT == 0);
    for (uint32_t q = 0; q < nr; ++q) lin &= a.rd[q].logT == 0;
    if (lin) plain ? reduce_slot_dispatch<true, true>(p.slot_cols, grid, p.lds, stream, a)
                   : reduce_slot_dispatch<true, false>(p.slot_cols, grid, p.lds, stream, a);
    else plain ? reduce_slot_dispatch<false, true>(p.slot_cols, grid, p.lds, stream, a)
               : reduce_slot_dispatch<false, false>(p.slot_cols, grid, p.lds, stream, a);
  } else if (f32 && KR >= 1) {
    bool lin = l.nbytes <= (1ull << 32) && (sec.key < 0 || a.key.logT == 0);
    for (uint32_t q = 0; q < nr; ++q) lin &= a.rd[q].logT == 0;
    if (lin) plain ? reduce_f32_dispatch<true, true>(KR, grid, stream, a) : reduce_f32_dispatch<true, false>(KR, grid, stream, a);
    else plain ? reduce_f32_dispatch<false, true>(KR, grid, stream, a) : reduce_f32_dispatch<false, false>(KR, grid, stream, a);
  } else if (w8) {
    plain ? reduce_dispatch<true, true>(KR, nr, grid, p.lds, stream, a) : reduce_dispatch<true, false>(KR, nr, grid, p.lds, stream, a);
  } else {
    plain ? reduce_dispatch<false, true>(KR, nr, grid, p.lds, stream, a) : reduce_dispatch<false, false>(KR, nr, grid, p.lds, stream, a);
  }
  hipError_t e = hipGetLastError();
  if (e == hipSuccess) {
    if (plain)
      hipLaunchKernelGGL(reduce_final_kernel<true>, dim3(a.cells), dim3(256), 0, stream, (const uint64_t *)partials,
                         p.groups, cols, a.fp_mask, (uint64_t *)out);
    else
      hipLaunchKernelGGL(reduce_final_kernel<false>, dim3(a.cells), dim3(256), 0, stream, (const uint64_t *)partials,
                         p.groups, cols, a.fp_mask, (uint64_t *)out);
    e = hipGetLastError();
  }
  if (e != hipSuccess) return fail(ADHA_ERR_DEVICE, "reduction launch failed: %s", hipGetErrorString(e));
  return ADHA_OK;
}

// Division by d >= 1 of any r < 2^31 as (r * m) >> s: with l = ceil(log2 d),
// m = ceil(2^(31+l) / d) < 2^32 and s = 31 + l.  m / 2^s exceeds 1/d by less
// than 2^-(31+l), so r * m / 2^s exceeds r / d by less than 2^-l <= 1/d,
// which never carries past the next integer: the floor is r / d exactly.
static void magic_div(uint32_t d, uint32_t *m, uint32_t *s) {
  uint32_t l = 0;
  while ((uint64_t(1) << l) < d) ++l;
  *m = (uint32_t)(((uint64_t(1) << (31 + l)) + d - 1) / d);
  *s = 31 + l;
}

// A reduction over no records writes a table of zeros.
__global__ void zero_u64_kernel(uint64_t *p, uint32_t n) {
  const uint32_t i = blockIdx.x * 256u + threadIdx.x;
  if (i < n) p[i] = 0;
}

adha_status section_launch(Ctx *ctx, const SectionDesc &sec, const LayoutDesc &l, void *buf,
                           const int32_t *idx, hipStream_t stream, void *out_override, void *scratch) {
  const int64_t n = l.shape.n;
  if (sec.op == ADHA_OP_REDUCE) {
    void *out = out_override ? out_override : sec.out;
    if (n == 0) {
      hipLaunchKernelGGL(zero_u64_kernel, dim3((sec.reduce_cells() + 255) / 256), dim3(256), 0, stream,
                         (uint64_t *)out, sec.reduce_cells());
      ADHA_HIP(hipGetLastError());
      return ADHA_OK;
    }
    if (!scratch) {
      ADHA_TRY(ctx_reduce_scratch(ctx));
      scratch = ctx->reduce_partials;
    }
    return reduce_launch(ctx, sec, l, buf, out, (uint64_t *)scratch, kReducePartialPairs * 16ull, stream);
  }
  if (n == 0) return ADHA_OK;
  SectionArgs a{};
  a.buf = (uint8_t *)buf;
  a.idx = idx;
  a.err = ctx->err_flag;
  a.n = n;
  a.degree = sec.degree;
  a.n_read = (uint32_t)sec.rd.size();
  a.n_write = (uint32_t)sec.wr.size();
  a.op = (uint32_t)sec.op;
  for (size_t q = 0; q < sec.rd.size(); ++q) a.rd[q] = sfield(l, sec.rd[q]);
  for (size_t k = 0; k < sec.wr.size(); ++k) a.wr[k] = sfield(l, sec.wr[k]);
  if (sec.stencil) {
    a.stencil = 1;
    a.nx = sec.nx;
    a.ny = sec.ny;
    a.nz = sec.nz;
    magic_div(sec.nx, &a.mx, &a.sx);
    magic_div(sec.ny, &a.my, &a.sy);
    for (uint32_t j = 0; j < sec.degree; ++j) {
      for (int c = 0; c < 3; ++c) a.off[j][c] = sec.offsets[3 * j + c];
      a.lin[j] = a.off[j][0] + (int32_t)sec.nx * (a.off[j][1] + (int32_t)sec.ny * a.off[j][2]);
    }
  }
  const dim3 grid((uint32_t)((n + 255) / 256));
  const uint32_t nr = a.n_read;
  // a read field narrower than 4 bytes or not 4-byte aligned: the byte-wise
  // form.  Narrow or unaligned write fields alone keep the dword loads: the
  // generic, span and generic-fold stencil kernels store through store_acc,
  // which writes such fields byte by byte; the straight-line forms below
  // (dword stores) are then left out.
  bool sub_rd = false, sub_wr = false;
  for (uint32_t q = 0; q < nr; ++q) sub_rd |= !a.rd[q].al;
  for (uint32_t k = 0; k < a.n_write; ++k) sub_wr |= !a.wr[k].al;
  auto wclass = [](uint32_t dt) { return dt == ADHA_F32 ? 0 : dt == ADHA_F64 ? 1 : 2; };
  const int wt0 = wclass(a.wr[0].dt), wt1 = a.n_write > 1 ? wclass(a.wr[1].dt) : 3;
  // a stencil with a narrow or unaligned read field, up to 8 reads: the fold
  // specialised on the write types.  (With aligned reads the linear-offset
  // forms below are faster, even with the generic fold.)
  if (sec.stencil && nr <= 8 && sub_rd && !ctx->no_span) {
    const bool lin = stencil_linear(a, l);
    bool w8 = false;
    for (uint32_t q = 0; q < nr; ++q) w8 |= a.rd[q].e == 8;
    if (nr <= 4) {
      if (!lin) launch_stencil_mixed<4, false, true>(wt0, wt1, grid, a, stream);
      else if (w8) launch_stencil_mixed<4, true, true>(wt0, wt1, grid, a, stream);
      else launch_stencil_mixed<4, true, false>(wt0, wt1, grid, a, stream);
    } else {
      if (!lin) launch_stencil_mixed<8, false, true>(wt0, wt1, grid, a, stream);
      else if (w8) launch_stencil_mixed<8, true, true>(wt0, wt1, grid, a, stream);
      else launch_stencil_mixed<8, true, false>(wt0, wt1, grid, a, stream);
    }
    ADHA_HIP(hipGetLastError());
    return ADHA_OK;
  }
  // a direct GEN / SUM section with a narrow or unaligned field: the mixed
  // direct kernel's narrow form
  if ((sec.op == ADHA_OP_GEN || sec.op == ADHA_OP_SUM) && sec.degree == 0 && !sec.stencil && (sub_rd || sub_wr) &&
      nr <= 16 && !ctx->no_span) {
    if (nr <= 4) launch_direct_mixed_w0<4, true, true>(wt0, wt1, a, stream);
    else launch_direct_mixed_w0<16, true, true>(wt0, wt1, a, stream);
    ADHA_HIP(hipGetLastError());
    return ADHA_OK;
  }
  if (sub_rd) {
    launch_sub(sec, nr, grid, a, stream);
    ADHA_HIP(hipGetLastError());
    return ADHA_OK;
  }
  // direct GEN / SUM over F32 fields only: the straight-line kernel
  bool all_f32 = true, all_t1 = l.nbytes <= (1ull << 32);
  for (uint32_t q = 0; q < nr; ++q) {
    all_f32 &= a.rd[q].dt == ADHA_F32;
    all_t1 &= a.rd[q].logT == 0;
  }
  for (uint32_t k = 0; k < a.n_write; ++k) all_f32 &= a.wr[k].dt == ADHA_F32;
  all_f32 &= !sub_wr;
  // direct GEN / SUM over F32, F64, I32 and U32 fields (not all F32): the
  // fold specialised on the write types, terms converted by selects
  bool wide_types = true, w8 = false;
  for (uint32_t q = 0; q < nr; ++q) {
    const uint32_t dt = a.rd[q].dt;
    wide_types &= dt == ADHA_F32 || dt == ADHA_F64 || dt == ADHA_I32 || dt == ADHA_U32;
    w8 |= a.rd[q].e == 8;
  }
  for (uint32_t k = 0; k < a.n_write; ++k) {
    const uint32_t dt = a.wr[k].dt;
    wide_types &= dt == ADHA_F32 || dt == ADHA_F64 || dt == ADHA_I32 || dt == ADHA_U32;
  }
  wide_types &= !sub_wr;
  if ((sec.op == ADHA_OP_GEN || sec.op == ADHA_OP_SUM) && sec.degree == 0 && !sec.stencil && !all_f32 &&
      wide_types && nr <= 16 && !ctx->no_span) {
    if (nr <= 4) w8 ? launch_direct_mixed_w0<4, true>(wt0, wt1, a, stream) : launch_direct_mixed_w0<4, false>(wt0, wt1, a, stream);
    else w8 ? launch_direct_mixed_w0<16, true>(wt0, wt1, a, stream) : launch_direct_mixed_w0<16, false>(wt0, wt1, a, stream);
    ADHA_HIP(hipGetLastError());
    return ADHA_OK;
  }
  if ((sec.op == ADHA_OP_GEN || sec.op == ADHA_OP_SUM) && sec.degree == 0 && !sec.stencil && all_f32) {
    if (all_t1) launch_direct_f32<true>(nr, grid, a, stream);
    else launch_direct_f32<false>(nr, grid, a, stream);
    ADHA_HIP(hipGetLastError());
    return ADHA_OK;
  }
  switch (sec.op) {
    case ADHA_OP_GEN: {
      if (sec.stencil) {
        bool w8 = false, f32 = true;
        const bool lin = stencil_linear(a, l);
        for (uint32_t q = 0; q < nr; ++q) {
          w8 |= a.rd[q].e == 8;
          f32 &= a.rd[q].dt == ADHA_F32;
        }
        for (uint32_t k = 0; k < a.n_write; ++k) f32 &= a.wr[k].dt == ADHA_F32;
        f32 &= !sub_wr;  // the F32 forms store dwords
        if (f32) {
          if (lin) launch_stencil<false, true, true>(nr, grid, a, stream);
          else launch_stencil<false, false, true>(nr, grid, a, stream);
        } else if (w8) {
          if (lin) launch_stencil<true, true, false>(nr, grid, a, stream);
          else launch_stencil<true, false, false>(nr, grid, a, stream);
        } else {
          if (lin) launch_stencil<false, true, false>(nr, grid, a, stream);
          else launch_stencil<false, false, false>(nr, grid, a, stream);
        }
        break;
      }
      SpanArgs sp{};
      uint32_t vec = 0;
      if (sec.degree > 0 && !ctx->no_span && span_plan(sec, l, &sp, &vec)) {
        if (vec == 16) launch_span<16>(nr, grid, a, sp, stream);
        else if (vec == 8) launch_span<8>(nr, grid, a, sp, stream);
        else launch_span<4>(nr, grid, a, sp, stream);
        break;
      }
      if (sec.degree == 0) launch_maxr<ADHA_OP_GEN, 0>(nr, grid, a, stream);
      else if (sec.degree <= 8) launch_maxr<ADHA_OP_GEN, 8>(nr, grid, a, stream);
      else if (sec.degree <= 16) launch_maxr<ADHA_OP_GEN, 16>(nr, grid, a, stream);
      else launch_maxr<ADHA_OP_GEN, 32>(nr, grid, a, stream);
      break;
    }
    case ADHA_OP_SUM:
      launch_maxr<ADHA_OP_SUM, 0>(nr, grid, a, stream);
      break;
    case ADHA_OP_MULADD3:
      hipLaunchKernelGGL((section_kernel<ADHA_OP_MULADD3, 0, 4, true>), grid, dim3(256), 0, stream, a);
      break;
    case ADHA_OP_SUB2:
      hipLaunchKernelGGL((section_kernel<ADHA_OP_SUB2, 0, 4, true>), grid, dim3(256), 0, stream, a);
      break;
    default:
      return fail(ADHA_ERR_UNSUPPORTED, "unknown op %d", sec.op);
  }
  ADHA_HIP(hipGetLastError());
  return ADHA_OK;
}

// ------------------------------------------------------------ static scratch
// Reduction partials for adha_section_run_static, which allocates nothing: a
// file-scope device array (16 MiB, the most any reduction's pass 1 writes).
// Each GPU the library runs on holds its own copy until the process ends,
// and every call on that GPU shares it.  Host code never passes the array's
// name (a host-side stand-in); it uses the device address looked up below.
static __device__ __align__(256) uint64_t scratch[kReducePartialPairs * 2];

adha_status static_scratch_address(int device, void **out) {
  static std::mutex m;
  static std::map<int, void *> addr;  // per device
  std::lock_guard<std::mutex> lk(m);
  auto it = addr.find(device);
  if (it == addr.end()) {
    DeviceGuard g(device);
    int cur = -1;
    if (hipGetDevice(&cur) != hipSuccess || cur != device)
      return fail(ADHA_ERR_DEVICE, "cannot make device %d current for its scratch array", device);
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
      return fail(ADHA_ERR_DEVICE, "hipGetSymbolAddress(scratch) on device %d failed: %s", device,
                  hipGetErrorString(e));
    it = addr.emplace(device, p).first;
  }
  *out = it->second;
  return ADHA_OK;
}

// Uniform neighbour indices in [0, n) for timing gather sections when the
// caller supplies none: SplitMix64 of the element index, multiply-shift.
__global__ void fill_uniform_index_kernel(int32_t *idx, uint64_t count, uint64_t n, uint64_t seed) {
  for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (uint64_t)gridDim.x * blockDim.x) {
    uint64_t z = (seed + i + 1) * 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    z ^= z >> 31;
    idx[i] = (int32_t)(((z >> 32) * n) >> 32);
  }
}

adha_status fill_uniform_index(int32_t *idx, uint64_t count, int64_t n, uint64_t seed, hipStream_t stream) {
  if (count == 0) return ADHA_OK;
  if (n <= 0 || n > (int64_t(1) << 31)) return fail(ADHA_ERR_INVALID, "index range %lld", (long long)n);
  const uint64_t blocks = std::min<uint64_t>((count + 255) / 256, 65536);
  hipLaunchKernelGGL(fill_uniform_index_kernel, dim3((uint32_t)blocks), dim3(256), 0, stream, idx, count,
                     (uint64_t)n, seed << 32);
  ADHA_HIP(hipGetLastError());
  return ADHA_OK;
}

}  // namespace adha
