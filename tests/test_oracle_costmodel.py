"""Pins for the oracle's analytic cost model (CPU only), host parity of the
library's analytic tables with it, and the library's cost-model features
against values worked out by hand."""
import ctypes
import math

import numpy as np
import pytest

from oracle import costmodel as OC
from oracle import planner as OP
from oracle.layout import Layout, aos, soa, from_partition
from paper_1407_4859_amd import adha as A
from paper_1407_4859_amd import synth


def test_bytes_by_hand():
    eb = [4, 4, 4, 8, 4]                     # S = 24
    n = 1 << 16
    # SoA, direct: only touched columns move
    assert OC.bytes_per_record([0, 1], [2], 0, soa(n, eb)) == 12.0
    # AoS, direct: one field of a 24-byte record drags the whole line, capped at S
    assert OC.bytes_per_record([0], [], 0, aos(n, eb)) == 24.0
    # tiled by 64: 4-byte columns of 256 bytes are dense
    assert OC.bytes_per_record([0, 3], [4], 0, Layout(n, eb, [0] * 5, [64])) == 16.0
    # tiled by 4: a 16-byte column piece drags a whole 128-byte line (32 per field), capped at S
    assert OC.bytes_per_record([0], [], 0, Layout(n, eb, [0] * 5, [4])) == 24.0
    # tiled by 16: a 64-byte column piece costs 128 / 16 = 8 bytes per record per field
    assert OC.bytes_per_record([0, 1], [], 0, Layout(n, eb, [0] * 5, [16])) == 16.0
    # gather, d = 2: SoA costs (e + 127) per field per neighbour plus 4 index bytes each
    assert OC.bytes_per_record([0, 3], [4], 2, soa(n, eb)) == 2 * (131 + 135) + 4 + 8
    # gather on AoS: span of fields 0..3 (bytes 0..20) + 127 per neighbour; the
    # write streams the 24-byte records
    assert OC.bytes_per_record([0, 3], [4], 2, aos(n, eb)) == 2 * (20 + 127) + 24 + 8


def test_library_features_by_hand():
    """The library's 16 features of a few (section, layout) pairs, worked out
    by hand from their definition in the library's header."""
    eb = [4, 4, 4, 8, 4]
    n = 1 << 18
    st = A.Struct(n, [A.F32, A.F32, A.F32, A.F64, A.F32], eb)
    sec = A.Section(st, A.OP_GEN, [0, 3], [4], 16)
    f = np.array(sec.features(A.Layout.soa(st)), np.float32)
    # SoA: both reads and the write sit in one-field groups; the gathered
    # footprint is N * (4 + 8) bytes; effective bytes 16 * (131 + 135) + 4 + 64
    want = [18 / 24, 2 / 16, 1 / 2, 16 / 32, math.log2(13) / 8, math.log2(5) / 8,
            2 / 16, 1 / 2, 0.0, 0.0, 1, 0, 0, 0, math.log2(12 * n) / 32,
            math.log2(16 * (131 + 135) + 4 + 64) / 12]
    assert np.array_equal(f, np.array(want, np.float64).astype(np.float32))
    # one group tiled by 64 holds everything: reads tiled, write in a
    # several-field group, footprint N * 24 bytes
    t = np.array(sec.features(A.Layout.create(st, [0] * 5, [64])), np.float32)
    assert list(t[10:15]) == [0, 0, 1, 1, np.float32(math.log2(24 * n) / 32)]
    # a direct section has no gathered footprint
    d = A.Section(st, A.OP_GEN, [0, 3], [4], 0)
    assert d.features(A.Layout.soa(st))[14] == 0
    # reads {0, 3} in the interleaved group {0..3} (20-byte records, so 4-byte
    # loads): the span runs over bytes 0..20, five loads per neighbour
    L = A.Layout.create(st, [0, 0, 0, 0, 1], [1, 1])
    g = np.array(sec.features(L), np.float32)
    assert g[8] == 1.0 and g[9] == np.float32(5 / 16)
    assert g[6] == np.float32(1 / 16) and list(g[10:14]) == [0, 1, 0, 0]
    assert g[14] == np.float32(math.log2(20 * n) / 32)
    # the same group tiled: no span loads
    g2 = np.array(sec.features(A.Layout.create(st, [0, 0, 0, 0, 1], [64, 1])), np.float32)
    assert g2[8] == 0 and g2[9] == 0
    # a direct section never takes the span path
    assert d.features(L)[8] == 0
    # layouts that differ only in groups the section does not touch give the
    # same features
    st7 = A.Struct(n, [A.F32] * 7, [4] * 7)
    s7 = A.Section(st7, A.OP_GEN, [0, 1], [2], 8)
    a1 = A.Layout.create(st7, [0, 0, 1, 2, 2, 3, 3], [1, 1, 1, 1])
    a2 = A.Layout.create(st7, [0, 0, 1, 2, 3, 4, 5], [1] * 6)
    assert s7.features(a1) == s7.features(a2)
    assert OC.layout_class(aos(n, eb)) == 0 and OC.layout_class(soa(n, eb)) == 1
    assert OC.layout_class(Layout(n, eb, [0] * 5, [64])) == 2
    assert OC.layout_class(from_partition(n, eb, [[0, 1]], 1)) == 3
    assert OC.layout_class(from_partition(n, eb, [[0, 1]], 64)) == 2


def test_library_analytic_tables_match_oracle():
    spec = synth.config3_struct(1 << 20)
    secs = synth.random_program(11, spec.n_fields)
    st = A.Struct.from_spec(spec)
    ss = [A.Section.from_spec(st, s) for s in secs]
    prog = A.Program(st, ss)
    opts = A.plan_opts(cost=A.COST_ANALYTIC, cap_bytes=128)
    h = ctypes.c_void_p()
    A.check(A.lib().adha_plan_create(None, prog.h, ctypes.byref(opts), None, 0, None, ctypes.byref(h)))
    pl = A.Plan(h, len(secs))
    osecs = [(s.read, s.write, s.degree) for s in secs]
    cat = OP.catalogue(osecs, spec.n, spec.elem_bytes, 128)
    T, R = pl.tables()
    for s, sec in enumerate(secs):
        for c, O in enumerate(cat):
            assert T[s][c] == pytest.approx(OC.section_us(sec.read, sec.write, sec.degree, O), rel=1e-12)
    for a, Oa in enumerate(cat):
        for b, Ob in enumerate(cat):
            assert R[a][b] == pytest.approx(OC.remap_us(Oa, Ob), rel=1e-12)
    for sec, s in zip(ss, secs):
        for c in range(0, len(cat), 5):
            assert sec.effective_bytes(pl.candidate(c)) == pytest.approx(
                spec.n * OC.bytes_per_record(s.read, s.write, s.degree, cat[c]), rel=1e-12)
