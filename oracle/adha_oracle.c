/*
 * CPU oracle for the data-layout hot path.  TEST INFRASTRUCTURE ONLY: it is
 * linked or called by the tests, by the smoke check and by the benchmark's
 * CPU-baseline leg, never by the library.  It shares no source with the
 * library and is deliberately plain: one record and one field at a time,
 * in the order the definitions state.  Build: gcc -O2 -ffp-contract=off
 * (no fast-math), so every floating-point operation rounds once, in IEEE
 * round-to-nearest-even, in the type the definition names.
 *
 * A layout is passed as one row per field of five uint64 values
 *   (base_g, T_g, S_g, p_f, e_f)
 * and the byte address of field f of record r is
 *   base_g + (r / T_g) * T_g * S_g + p_f * T_g + (r % T_g) * e_f.
 * The rows are produced by the oracle's own layout module.
 */
#include <stdint.h>
#include <string.h>

enum { ORC_F32 = 0, ORC_F64 = 1, ORC_I32 = 2, ORC_RAW = 3, ORC_U32 = 4, ORC_U8 = 5, ORC_U16 = 6, ORC_I16 = 7 };
enum { ORC_GEN = 0, ORC_MULADD3 = 1, ORC_SUB2 = 2, ORC_SUM = 3 };

#define ORC_MAX_TERMS 1024

static uint64_t orc_addr(const uint64_t *row, uint64_t r)
{
    uint64_t base = row[0], t = row[1], s = row[2], p = row[3], e = row[4];
    return base + (r / t) * t * s + p * t + (r % t) * e;
}

uint64_t orc_layout_addr(const uint64_t *desc, int32_t f, int64_t r)
{
    return orc_addr(desc + 5 * (int64_t)f, (uint64_t)r);
}

/*
 * Remap (section 2: the remap edge and its operation; section 3, the
 * Medical program's remap between its CPU and GPU sections): every field of
 * every record in [r_begin, r_end) is copied from its source address to its
 * destination address.  The destination's padding is the caller's business
 * (it starts from a zero-filled buffer).
 */
void orc_remap(int32_t n_fields, const uint64_t *src_desc, const uint8_t *src,
               const uint64_t *dst_desc, uint8_t *dst, int64_t r_begin, int64_t r_end)
{
    for (int64_t r = r_begin; r < r_end; ++r)
        for (int32_t f = 0; f < n_fields; ++f) {
            const uint64_t *sr = src_desc + 5 * f, *dr = dst_desc + 5 * f;
            memcpy(dst + orc_addr(dr, (uint64_t)r), src + orc_addr(sr, (uint64_t)r), (size_t)sr[4]);
        }
}

/* ---------------------------------------------------------------- sections */

typedef struct {
    int32_t dt;
    uint64_t bits; /* little-endian element bytes, zero-extended */
} orc_term;

static orc_term orc_load(const uint8_t *buf, const uint64_t *row, int32_t dt, uint64_t r)
{
    orc_term t;
    t.dt = dt;
    t.bits = 0;
    memcpy(&t.bits, buf + orc_addr(row, r), (size_t)row[4]);
    return t;
}

/*
 * Integer element types: I32 and I16 are two's complement, U32, U16 and U8
 * unsigned; t.bits holds the element's bytes zero-extended.  As a number an
 * integer term is its mathematical value; converting it to a floating-point
 * type rounds to nearest even (exact below 2^24 for float, always for
 * double).  As 32 bits (the integer fold) it is that value modulo 2^32, so
 * I16 is sign-extended and the unsigned types zero-extended.
 */
static int64_t orc_int_value(orc_term t)
{
    switch (t.dt) {
    case ORC_I32: return (int32_t)(uint32_t)t.bits;
    case ORC_I16: return (int16_t)(uint16_t)t.bits;
    case ORC_U32: return (uint32_t)t.bits;
    case ORC_U16: return (uint16_t)t.bits;
    default: return (uint8_t)t.bits;
    }
}

static float orc_to_f32(orc_term t)
{
    if (t.dt == ORC_F32) { float v; uint32_t b = (uint32_t)t.bits; memcpy(&v, &b, 4); return v; }
    if (t.dt == ORC_F64) { double v; memcpy(&v, &t.bits, 8); return (float)v; }
    return (float)orc_int_value(t);
}

static double orc_to_f64(orc_term t)
{
    if (t.dt == ORC_F32) { float v; uint32_t b = (uint32_t)t.bits; memcpy(&v, &b, 4); return (double)v; }
    if (t.dt == ORC_F64) { double v; memcpy(&v, &t.bits, 8); return v; }
    return (double)orc_int_value(t);
}

static uint32_t orc_bits32(orc_term t)
{
    if (t.dt == ORC_F64) return (uint32_t)t.bits ^ (uint32_t)(t.bits >> 32);
    if (t.dt == ORC_F32) return (uint32_t)t.bits;
    return (uint32_t)(uint64_t)orc_int_value(t);
}

/*
 * One section (section 2: a section is one data-parallel loop; the paper
 * gives no loop bodies, so the bodies are the ones the workloads define):
 * for every record i in [r_begin, r_end) the terms are read first -- direct
 * (degree 0): the read fields at i in ascending id; gather: for j = 0..d-1
 * the read fields, in ascending id, of record idx[i*d + j] -- and then each
 * write field w_k (ascending id) is written at i:
 *   GEN, fp w:  acc = 0; per term v = convert(t) to w's type;
 *               k = 0: acc = acc + v;  k = 1: acc = acc*0.5 + v
 *   GEN, integer w: acc = 0 (mod 2^32); per term u = its 32 bits (fp64: low ^
 *               high; an integer term's value modulo 2^32);
 *               k = 0: acc = acc + u;  k = 1: acc = (acc ^ u) * 16777619;
 *               stored as the low bytes of acc that fit w
 *   MULADD3: w = a*b + c;  SUB2: w = a - b;  SUM: w = ((t0 + t1) + ...)
 * with a, b, c the three read fields in ascending id, each converted to w's
 * type first.  Returns the number of gather indices outside [0, n).
 */
int64_t orc_section(int32_t op, int64_t n, const uint64_t *desc, const int32_t *dtypes,
                    int32_t n_read, const int32_t *rd, int32_t n_write, const int32_t *wr,
                    int32_t degree, const int32_t *idx, uint8_t *buf,
                    int64_t r_begin, int64_t r_end)
{
    orc_term terms[ORC_MAX_TERMS];
    int64_t bad = 0;
    int32_t per = degree > 0 ? degree * n_read : n_read;
    if (per > ORC_MAX_TERMS) return -1;
    for (int64_t i = r_begin; i < r_end; ++i) {
        int32_t nt = 0;
        if (degree == 0) {
            for (int32_t q = 0; q < n_read; ++q)
                terms[nt++] = orc_load(buf, desc + 5 * rd[q], dtypes[rd[q]], (uint64_t)i);
        } else {
            for (int32_t j = 0; j < degree; ++j) {
                int32_t nb = idx[i * degree + j];
                if (nb < 0 || nb >= n) { ++bad; continue; }
                for (int32_t q = 0; q < n_read; ++q)
                    terms[nt++] = orc_load(buf, desc + 5 * rd[q], dtypes[rd[q]], (uint64_t)nb);
            }
        }
        for (int32_t k = 0; k < n_write; ++k) {
            int32_t w = wr[k];
            int32_t wdt = dtypes[w];
            uint8_t *dst = buf + orc_addr(desc + 5 * w, (uint64_t)i);
            if (wdt == ORC_F32) {
                float acc = 0.0f;
                if (op == ORC_MULADD3) {
                    float a = orc_to_f32(terms[0]), b = orc_to_f32(terms[1]), c = orc_to_f32(terms[2]);
                    float ab = a * b;
                    acc = ab + c;
                } else if (op == ORC_SUB2) {
                    acc = orc_to_f32(terms[0]) - orc_to_f32(terms[1]);
                } else {
                    for (int32_t q = 0; q < nt; ++q) {
                        float v = orc_to_f32(terms[q]);
                        if (op == ORC_GEN && k == 1) { float h = acc * 0.5f; acc = h + v; }
                        else acc = acc + v;
                    }
                }
                memcpy(dst, &acc, 4);
            } else if (wdt == ORC_F64) {
                double acc = 0.0;
                if (op == ORC_MULADD3) {
                    double a = orc_to_f64(terms[0]), b = orc_to_f64(terms[1]), c = orc_to_f64(terms[2]);
                    double ab = a * b;
                    acc = ab + c;
                } else if (op == ORC_SUB2) {
                    acc = orc_to_f64(terms[0]) - orc_to_f64(terms[1]);
                } else {
                    for (int32_t q = 0; q < nt; ++q) {
                        double v = orc_to_f64(terms[q]);
                        if (op == ORC_GEN && k == 1) { double h = acc * 0.5; acc = h + v; }
                        else acc = acc + v;
                    }
                }
                memcpy(dst, &acc, 8);
            } else {
                /* an integer write field: the fold modulo 2^32, stored as its
                   low e bytes (the value modulo 2^(8e)) */
                uint32_t acc = 0;
                for (int32_t q = 0; q < nt; ++q) {
                    uint32_t u = orc_bits32(terms[q]);
                    if (k == 1) acc = (acc ^ u) * 16777619u;
                    else acc = acc + u;
                }
                uint8_t le[4] = {(uint8_t)acc, (uint8_t)(acc >> 8), (uint8_t)(acc >> 16), (uint8_t)(acc >> 24)};
                memcpy(dst, le, (size_t)desc[5 * w + 4]);
            }
        }
    }
    return bad;
}
