"""Pins for the oracle's analytic cost model and features (CPU only), and
host parity of the library's analytic tables and features with them."""
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
    # AoS, direct: one field of a 24-byte record costs a granule, capped at S
    assert OC.bytes_per_record([0], [], 0, aos(n, eb)) == 24.0
    # tiled by 64: 4-byte columns of 256 bytes are dense
    assert OC.bytes_per_record([0, 3], [4], 0, Layout(n, eb, [0] * 5, [64])) == 16.0
    # tiled by 4: a 16-byte column piece drags a whole granule (16 per field), capped
    assert OC.bytes_per_record([0], [], 0, Layout(n, eb, [0] * 5, [4])) == 16.0
    # gather, d = 2: SoA costs (e + 63) per field per neighbour plus 4 index bytes each
    assert OC.bytes_per_record([0, 3], [4], 2, soa(n, eb)) == 2 * (67 + 71) + 4 + 8
    # gather on AoS: span of fields 0..3 (bytes 0..20) + 63 per neighbour
    assert OC.bytes_per_record([0, 3], [4], 2, aos(n, eb)) == 2 * (20 + 63) + 24 + 8


def test_features_by_hand():
    eb = [4, 4, 4, 8, 4]
    n = 1 << 18
    f = OC.features([0, 3], [4], 16, soa(n, eb))
    # SoA: both reads and the write sit in one-field groups; the gathered
    # footprint is N * (4 + 8) bytes
    want = [18 / 24, 2 / 16, 1 / 2, 16 / 32, math.log2(13) / 8, math.log2(5) / 8,
            2 / 16, 1 / 2, 0.0, 0.0, 1, 0, 0, 0, math.log2(12 * n) / 32,
            math.log2(16 * (67 + 71) + 4 + 64) / 12]
    assert np.array_equal(f, np.array(want, np.float64).astype(np.float32))
    # one group tiled by 64 holds everything: reads tiled, write in a
    # several-field group, footprint N * 24 bytes
    t = OC.features([0, 3], [4], 16, Layout(n, eb, [0] * 5, [64]))
    assert list(t[10:15]) == [0, 0, 1, 1, np.float32(math.log2(24 * n) / 32)]
    # a direct section has no gathered footprint
    assert OC.features([0, 3], [4], 0, soa(n, eb))[14] == 0
    # reads {0, 3} in the interleaved group {0..3} (20-byte records, so 4-byte
    # loads): the span runs over bytes 0..20, five loads per neighbour
    L = from_partition(n, eb, [[0, 1, 2, 3]], 1)
    g = OC.features([0, 3], [4], 16, L)
    assert OC.span_loads([0, 3], 16, L) == 5 and g[8] == 1.0 and g[9] == np.float32(5 / 16)
    assert g[6] == np.float32(1 / 16) and list(g[10:14]) == [0, 1, 0, 0]
    assert g[14] == np.float32(math.log2(20 * n) / 32)
    assert OC.span_loads([0, 3], 0, L) == 0                               # direct
    assert OC.span_loads([0, 3], 16, from_partition(n, eb, [[0, 1, 2, 3]], 64)) == 0  # tiled
    # 32-byte records with 16-byte loads: reads at bytes 20..28 need one load at 16..32
    eb2 = [4, 4, 4, 4, 4, 8, 4]
    L2 = from_partition(n, eb2, [[0, 1, 2, 3, 4, 5, 6]], 1)
    assert OC.span_loads([5], 4, L2) == 1 and OC.span_loads([0, 6], 4, L2) == 2
    assert OC.layout_class(aos(n, eb)) == 0 and OC.layout_class(soa(n, eb)) == 1
    assert OC.layout_class(Layout(n, eb, [0] * 5, [64])) == 2
    assert OC.layout_class(from_partition(n, eb, [[0, 1]], 1)) == 3
    assert OC.layout_class(from_partition(n, eb, [[0, 1]], 64)) == 2


def test_library_analytic_tables_and_features_match_oracle():
    spec = synth.config3_struct(1 << 20)
    secs = synth.random_program(11, spec.n_fields)
    st = A.Struct.from_spec(spec)
    ss = [A.Section.from_spec(st, s) for s in secs]
    prog = A.Program(st, ss)
    opts = A.plan_opts(cost=A.COST_ANALYTIC, cap_bytes=64)
    h = ctypes.c_void_p()
    A.check(A.lib().adha_plan_create(None, prog.h, ctypes.byref(opts), None, 0, None, ctypes.byref(h)))
    pl = A.Plan(h, len(secs))
    osecs = [(s.read, s.write, s.degree) for s in secs]
    cat = OP.catalogue(osecs, spec.n, spec.elem_bytes, 64)
    T, R = pl.tables()
    for s, sec in enumerate(secs):
        for c, O in enumerate(cat):
            assert T[s][c] == pytest.approx(OC.section_us(sec.read, sec.write, sec.degree, O), rel=1e-12)
    for a, Oa in enumerate(cat):
        for b, Ob in enumerate(cat):
            assert R[a][b] == pytest.approx(OC.remap_us(Oa, Ob), rel=1e-12)
    for sec, s in zip(ss, secs):
        for c in range(0, len(cat), 5):
            got = np.array(sec.features(pl.candidate(c)), np.float32)
            want = OC.features(s.read, s.write, s.degree, cat[c])
            assert np.array_equal(got, want)
            assert sec.effective_bytes(pl.candidate(c)) == pytest.approx(
                spec.n * OC.bytes_per_record(s.read, s.write, s.degree, cat[c]), rel=1e-12)
