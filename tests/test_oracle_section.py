"""Pins for the oracle's section semantics (CPU only)."""
import struct

import numpy as np
import pytest

import oracle
from oracle.layout import Layout, aos, soa, from_partition
from paper_1407_4859_amd import synth
from paper_1407_4859_amd.synth import F32, F64, I32, OP_GEN, OP_MULADD3, OP_SUB2, OP_SUM

FNV_PRIME = 16777619


def _cols(seed, st):
    return synth.record_matrix(seed, st.n, st.dtypes, st.elem_bytes)


def _as(col, dt):
    return col.view({F32: np.float32, F64: np.float64, I32: np.int32}[dt]).reshape(-1)


def _run_program(L, st, secs, cols, idx=None):
    buf = oracle.pack(L, cols)
    for s in secs:
        oracle.section(L, st.dtypes, s.op, s.read, s.write, s.degree,
                       idx if s.degree else None, buf)
    return [oracle.unpack(L, buf, f) for f in range(st.n_fields)]


@pytest.mark.parametrize("n", [1, 2, 1000])
def test_config1_sections_match_numpy_float32(n):
    st = synth.config1_struct(n)
    cols = _cols(1, st)
    out = _run_program(aos(n, st.elem_bytes), st, synth.config1_sections(), cols)
    x = [_as(c, F32).copy() for c in cols]
    x[3] = x[0] * x[1] + x[2]              # numpy float32: two roundings, no fusion
    x[5] = x[3] - x[4]
    x[7] = np.add.accumulate(np.stack(x[:7], axis=1), axis=1)[:, -1]   # sequential
    for f in range(8):
        assert np.array_equal(_as(out[f], F32).view(np.uint32), x[f].view(np.uint32)), f


def test_hand_case_n1():
    st = synth.config1_struct(1)
    vals = [2.0, 3.0, 1.0, 0.0, 0.5, 0.0, 0.25, 0.0]
    cols = [np.frombuffer(struct.pack("<f", v), np.uint8).reshape(1, 4).copy() for v in vals]
    out = _run_program(soa(1, st.elem_bytes), st, synth.config1_sections(), cols)
    got = [struct.unpack("<f", out[f].tobytes())[0] for f in range(8)]
    assert got[3] == 7.0 and got[5] == 6.5
    assert got[7] == 2.0 + 3.0 + 1.0 + 7.0 + 0.5 + 6.5 + 0.25


def test_muladd3_f64_matches_numpy():
    st = synth.StructSpec(500, [F64] * 4, [8] * 4)
    cols = _cols(9, st)
    out = _run_program(aos(500, st.elem_bytes), st,
                       [synth.SectionSpec(OP_MULADD3, [0, 1, 2], [3])], cols)
    x = [_as(c, F64) for c in cols]
    assert np.array_equal(_as(out[3], F64), x[0] * x[1] + x[2])


def test_layout_independence_config3_program():
    n = 600
    st = synth.config3_struct(n)
    cols = _cols(3, st)
    secs = synth.random_program(3, st.n_fields)
    idx = synth.uniform_index(3, 999, n * 16, n)
    layouts = [aos(n, st.elem_bytes), soa(n, st.elem_bytes),
               Layout(n, st.elem_bytes, [0] * 32, [64]),
               from_partition(n, st.elem_bytes, [[0, 5, 9], [28, 1, 20], [30, 31]], 1),
               from_partition(n, st.elem_bytes, [[0, 5, 9], [28, 1, 20], [30, 31]], 64)]
    ref = _run_program(layouts[0], st, secs, cols, idx)
    for L in layouts[1:]:
        got = _run_program(L, st, secs, cols, idx)
        for f in range(st.n_fields):
            assert np.array_equal(got[f], ref[f]), (L, f)
    # the program changed every written field
    written = {w for s in secs for w in s.write}
    assert any(not np.array_equal(ref[f], cols[f]) for f in written)


def test_gen_fp_k0_is_sequential_sum_and_conversions():
    # f32 output from an f32, an i32 (rounded to nearest even) and an f64 term
    st = synth.StructSpec(300, [F32, I32, F64, F32], [4, 4, 8, 4])
    cols = _cols(4, st)
    out = _run_program(aos(300, st.elem_bytes), st, [synth.SectionSpec(OP_GEN, [0, 1, 2], [3])],
                       cols)
    terms = np.stack([_as(cols[0], F32), _as(cols[1], I32).astype(np.float32),
                      _as(cols[2], F64).astype(np.float32)], axis=1)
    assert np.array_equal(_as(out[3], F32), np.add.accumulate(terms, axis=1)[:, -1])
    # int -> float rounds to nearest, ties to even
    st2 = synth.StructSpec(1, [I32, F32], [4, 4])
    c2 = [np.array([[1, 0, 0, 1]], np.uint8), np.zeros((1, 4), np.uint8)]  # 2^24 + 1
    o2 = _run_program(aos(1, st2.elem_bytes), st2, [synth.SectionSpec(OP_GEN, [0], [1])], c2)
    assert _as(o2[1], F32)[0] == np.float32(16777216.0)


def test_gen_fp_k1_is_halving_filter():
    # acc <- acc/2 + v on small integers is exact: acc = sum v_i 2^-(n-1-i)
    n, nr = 200, 9
    st = synth.StructSpec(n, [F32] * nr + [F32, F32], [4] * (nr + 2))
    z = synth.splitmix64(8, 0, 0, n * nr)
    v = ((z >> np.uint64(60)).astype(np.int64) - 8).astype(np.float32).reshape(n, nr)
    cols = [v[:, q].copy().view(np.uint8).reshape(n, 4) for q in range(nr)]
    cols += [np.zeros((n, 4), np.uint8)] * 2
    out = _run_program(soa(n, st.elem_bytes), st,
                       [synth.SectionSpec(OP_GEN, list(range(nr)), [nr, nr + 1])], cols)
    w = 2.0 ** -np.arange(nr - 1, -1, -1)
    assert np.array_equal(_as(out[nr + 1], F32).astype(np.float64), v.astype(np.float64) @ w)
    assert np.array_equal(_as(out[nr], F32), v.sum(axis=1))


def test_gen_int_outputs():
    n = 400
    st = synth.StructSpec(n, [I32, F32, F64, I32, I32], [4, 4, 8, 4, 4])
    cols = _cols(6, st)
    out = _run_program(aos(n, st.elem_bytes), st, [synth.SectionSpec(OP_GEN, [0, 1, 2], [3, 4])],
                       cols)
    d = _as(cols[2], F64).view(np.uint64)
    u = np.stack([_as(cols[0], I32).view(np.uint32), _as(cols[1], F32).view(np.uint32),
                  ((d & np.uint64(0xFFFFFFFF)) ^ (d >> np.uint64(32))).astype(np.uint32)], axis=1)
    # k = 0: wrapping sum of the 32-bit patterns
    k0 = (u.astype(np.uint64).sum(axis=1) % (1 << 32)).astype(np.uint32)
    assert np.array_equal(_as(out[3], I32).view(np.uint32), k0)
    # k = 1: undo the fold with the prime's inverse mod 2^32; it must end at 0
    inv = pow(FNV_PRIME, -1, 1 << 32)
    acc = _as(out[4], I32).view(np.uint32).astype(np.uint64)
    for q in range(2, -1, -1):
        acc = ((acc * np.uint64(inv)) % np.uint64(1 << 32)) ^ u[:, q].astype(np.uint64)
    assert not acc.any()
    # fp64 -> 32 bits is low word xor high word: 1.0 = 0x3FF00000_00000000
    assert struct.unpack("<II", struct.pack("<d", 1.0)) == (0, 0x3FF00000)


def test_gather_reduces_to_direct():
    n = 500
    st = synth.StructSpec(n, [F32, I32, F64, F32, I32], [4, 4, 8, 4, 4])
    cols = _cols(12, st)
    L = from_partition(n, st.elem_bytes, [[0, 2], [1, 3]], 1)
    direct = _run_program(L, st, [synth.SectionSpec(OP_GEN, [0, 1, 2], [3, 4])], cols)
    ident = np.arange(n, dtype=np.int32)
    g1 = _run_program(L, st, [synth.SectionSpec(OP_GEN, [0, 1, 2], [3, 4], 1)], cols, ident)
    assert all(np.array_equal(direct[f], g1[f]) for f in range(5))
    # a permutation gathers the direct result from the permuted record
    perm = np.argsort(synth.splitmix64(12, 51, 0, n)).astype(np.int32)
    gp = _run_program(L, st, [synth.SectionSpec(OP_GEN, [0, 1, 2], [3, 4], 1)], cols, perm)
    for f in (3, 4):
        assert np.array_equal(gp[f], direct[f][perm])
    # degree 2 with idx = [i, i] repeats the terms in order
    dup = np.repeat(ident, 2)
    g2 = _run_program(L, st, [synth.SectionSpec(OP_GEN, [0, 2], [3], 2)], cols, dup)
    t = np.stack([_as(cols[0], F32), _as(cols[2], F64).astype(np.float32)] * 2, axis=1)
    assert np.array_equal(_as(g2[3], F32), np.add.accumulate(t, axis=1)[:, -1])


def test_gather_out_of_range_index_is_skipped_and_counted():
    n = 10
    st = synth.StructSpec(n, [F32, F32], [4, 4])
    cols = _cols(13, st)
    L = soa(n, st.elem_bytes)
    idx = np.arange(n, dtype=np.int32)
    idx[3] = n
    idx[7] = -1
    buf = oracle.pack(L, cols)
    bad = oracle.section(L, st.dtypes, OP_GEN, [0], [1], 1, idx, buf)
    assert bad == 2
    got = _as(oracle.unpack(L, buf, 1), F32)
    assert got[3] == 0.0 and got[7] == 0.0
    assert got[0] == _as(cols[0], F32)[0]


def test_direct_section_reads_before_writing():
    # W overlaps R: every write uses the values read before any write
    n = 64
    st = synth.StructSpec(n, [F32, F32], [4, 4])
    cols = _cols(14, st)
    out = _run_program(aos(n, st.elem_bytes), st, [synth.SectionSpec(OP_GEN, [0, 1], [0, 1])],
                       cols)
    a, b = _as(cols[0], F32), _as(cols[1], F32)
    assert np.array_equal(_as(out[0], F32), a + b)
    assert np.array_equal(_as(out[1], F32), a * np.float32(0.5) + b)


# ---------------------------------------------------------------- narrow and unsigned integer fields
U32, U8, U16, I16 = oracle.U32, oracle.U8, oracle.U16, oracle.I16


def _col(vals, fmt):
    size = struct.calcsize("<" + fmt)
    return np.frombuffer(b"".join(struct.pack("<" + fmt, v) for v in vals), np.uint8).reshape(len(vals), size).copy()


def _run_one(dtypes, eb, cols, read, write, layout_of=None, op=OP_GEN):
    n = cols[0].shape[0]
    L = layout_of(n, eb) if layout_of else aos(n, eb)
    buf = oracle.pack(L, cols)
    oracle.section(L, dtypes, op, read, write, 0, None, buf)
    return [oracle.unpack(L, buf, f) for f in range(len(eb))]


def test_narrow_integers_convert_exactly_to_floating_point():
    """U8, U16, I16 terms are exact in float and double: a one-term GEN sum
    into an F32 and an F64 field gives the values back."""
    u8 = [0, 1, 127, 128, 255]
    u16 = [0, 1, 32768, 65534, 65535]
    i16 = [-32768, -1, 0, 1, 32767]
    for dt, fmt, vals, e in ((U8, "B", u8, 1), (U16, "H", u16, 2), (I16, "h", i16, 2)):
        cols = [_col(vals, fmt), _col([0.0] * 5, "f"), _col([0.0] * 5, "d")]
        out = _run_one([dt, F32, F64], [e, 4, 8], cols, [0], [1, 2])
        f32 = [struct.unpack("<f", out[1][r].tobytes())[0] for r in range(5)]
        f64 = [struct.unpack("<d", out[2][r].tobytes())[0] for r in range(5)]
        # write k = 1 folds acc*0.5 + v from acc = 0: the value itself
        assert f32 == [float(v) for v in vals] and f64 == [float(v) for v in vals], dt


def test_u32_rounds_to_nearest_even_in_float():
    """U32 is unsigned: 2^32 - 1 is 4294967295 (not -1); in float it rounds
    to nearest even (2^24 + 1 -> 2^24, 2^24 + 3 -> 2^24 + 4), in double it is
    exact."""
    vals = [4294967295, 16777217, 16777219, 2147483648, 7]
    cols = [_col(vals, "I"), _col([0.0] * 5, "f"), _col([0.0] * 5, "d")]
    out = _run_one([U32, F32, F64], [4, 4, 8], cols, [0], [1, 2])
    f32 = [struct.unpack("<f", out[1][r].tobytes())[0] for r in range(5)]
    f64 = [struct.unpack("<d", out[2][r].tobytes())[0] for r in range(5)]
    assert f32 == [4294967296.0, 16777216.0, 16777220.0, 2147483648.0, 7.0]
    assert f64 == [float(v) for v in vals]


def test_integer_fold_into_narrow_write_fields_keeps_the_low_bytes():
    """Worked by hand: the integer fold runs modulo 2^32 over the terms' 32-bit
    values (I16 sign-extended, unsigned types zero-extended) and a narrow
    write field keeps the low bytes."""
    # terms: I32 200, I16 -1 (0xFFFFFFFF), U16 65535 (0x0000FFFF), U8 100
    dtypes = [I32, I16, U16, U8, U8, U16, I16, U32]
    eb = [4, 2, 2, 1, 1, 2, 2, 4]
    cols = [_col([200], "i"), _col([-1], "h"), _col([65535], "H"), _col([100], "B"),
            _col([0], "B"), _col([0], "H"), _col([0], "h"), _col([0], "I")]
    # k = 0 sum: 200 + 0xFFFFFFFF + 0xFFFF + 100 = 0x1_0001_012A -> 0x0001012A
    s32 = (200 + 0xFFFFFFFF + 0xFFFF + 100) % (1 << 32)
    assert s32 == 0x0001012A
    for w, fmt, want in ((4, "B", s32 & 0xFF), (5, "H", s32 & 0xFFFF), (7, "I", s32)):
        out = _run_one(dtypes, eb, cols, [0, 1, 2, 3], [w])
        assert struct.unpack("<" + fmt, out[w][0].tobytes())[0] == want, w
    # an I16 write of 0x8000 reads back as -32768
    c2 = [_col([0x7FFF], "i"), _col([1], "h"), _col([0], "H"), _col([0], "B"),
          _col([0], "B"), _col([0], "H"), _col([0], "h"), _col([0], "I")]
    out = _run_one(dtypes, eb, c2, [0, 1], [6])
    assert struct.unpack("<h", out[6][0].tobytes())[0] == -32768
    # k = 1 (FNV fold) into a U32 and a U8 field: acc = (acc ^ u) * 16777619 mod 2^32
    acc = 0
    for u in (200, 0xFFFFFFFF, 0xFFFF, 100):
        acc = ((acc ^ u) * FNV_PRIME) % (1 << 32)
    out = _run_one(dtypes, eb, cols, [0, 1, 2, 3], [4, 7])
    assert struct.unpack("<I", out[7][0].tobytes())[0] == acc
    # the first write (k = 0) of the pair is the sum
    assert out[4][0][0] == s32 & 0xFF


def test_narrow_fields_are_layout_independent():
    """A struct of 1-, 2-, 4- and 8-byte typed fields (unaligned members in
    interleaved groups): a direct section and a gather give the same field
    bytes under every layout."""
    n = 257
    dtypes = [U8, I16, F32, U16, F64, U32, I32, U8, F32, I16]
    eb = [1, 2, 4, 2, 8, 4, 4, 1, 4, 2]
    cols = [synth.field_values(17, f, n, synth.RAW, e) for f, e in enumerate(eb)]
    idx = synth.uniform_index(17, 99, n * 4, n)
    secs = [synth.SectionSpec(OP_GEN, [0, 1, 2, 3, 4], [8, 9]), synth.SectionSpec(OP_GEN, [0, 3, 5, 6], [7], 4),
            synth.SectionSpec(OP_GEN, [1, 7, 9], [2, 5])]
    st = synth.StructSpec(n, dtypes, eb)
    outs = []
    for L in (aos(n, eb), soa(n, eb), Layout(n, eb, [0, 0, 0, 1, 1, 1, 2, 2, 2, 2], [1, 64, 4]),
              from_partition(n, eb, [[0, 1, 7, 9], [3, 5]], 1)):
        outs.append(_run_program(L, st, secs, cols, idx))
    for o in outs[1:]:
        for f in range(len(eb)):
            assert np.array_equal(o[f], outs[0][f]), f
