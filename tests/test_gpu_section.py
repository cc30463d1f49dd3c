"""GPU parity of the section kernels against the oracle (bit-exact expected,
the gate for floating-point outputs is 1 ulp)."""
import itertools

import numpy as np
import pytest
import torch

import oracle
from oracle.layout import Layout as OLayout, aos as oaos, soa as osoa, from_partition
from paper_1407_4859_amd import adha as A
from paper_1407_4859_amd import synth
from gpu_util import dev_bytes, host, mirror, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    return A.Ctx(0)


def ulp_distance(g: np.ndarray, w: np.ndarray, dt) -> float:
    """Largest distance in units in the last place between two fp columns
    (element bytes uint8 [n, e]); integer columns must match exactly."""
    if dt not in (synth.F32, synth.F64):
        return 0.0 if np.array_equal(g, w) else float("inf")
    it = np.int32 if dt == synth.F32 else np.int64
    x = g.copy().view(it).reshape(-1).astype(np.float64)
    y = w.copy().view(it).reshape(-1).astype(np.float64)
    top = float(np.iinfo(it).min)
    kx = np.where(x >= 0, x, top - x)     # sign-magnitude onto a monotone line
    ky = np.where(y >= 0, y, top - y)
    return float(np.max(np.abs(kx - ky))) if len(kx) else 0.0


def _compare(spec, O, got_buf, want_buf, fields, label):
    for f in fields:
        g = oracle.unpack(O, got_buf, f)
        w = oracle.unpack(O, want_buf, f)
        if not np.array_equal(g, w):
            u = ulp_distance(g, w, spec.dtypes[f])
            assert u <= 1, (label, f, u)


def _run_sections(ctx, spec, O, secs, cols, idx_h=None, label=""):
    st = A.Struct.from_spec(spec)
    L = mirror(st, O)
    buf_h = oracle.pack(O, cols)
    want = buf_h.copy()
    dev = dev_bytes(buf_h)
    idx = torch.from_numpy(idx_h).cuda() if idx_h is not None else None
    for s in secs:
        say("section", label, s, O)
        oracle.section(O, spec.dtypes, s.op, s.read, s.write, s.degree, idx_h, want)
        sec = A.Section.from_spec(st, s)
        A.section_run(ctx, sec, L, dev, idx if s.degree else None)
    ctx.check()
    got = host(dev, O.nbytes)
    _compare(spec, O, got, want, range(spec.n_fields), label)
    return got


@pytest.mark.parametrize("n", [1, 2, 255, 65536])
def test_config1_all_layout_combinations(ctx, n):
    spec = synth.config1_struct(n)
    cols = synth.record_matrix(1, n, spec.dtypes, spec.elem_bytes)
    secs = synth.config1_sections()
    st = A.Struct.from_spec(spec)
    lays = [oaos(n, spec.elem_bytes), osoa(n, spec.elem_bytes)]
    ref = None
    for combo in itertools.product(range(2), repeat=3):
        # run each section in its layout, remapping on the device in between
        cur = lays[combo[0]]
        buf = dev_bytes(oracle.pack(cur, cols))
        for s, c in zip(secs, combo):
            if lays[c] is not cur:
                nb = torch.empty(lays[c].nbytes, dtype=torch.uint8, device="cuda")
                A.remap(ctx, mirror(st, cur), buf, mirror(st, lays[c]), nb)
                buf, cur = nb, lays[c]
            A.section_run(ctx, A.Section.from_spec(st, s), mirror(st, cur), buf)
        ctx.check()
        out = [oracle.unpack(cur, host(buf, cur.nbytes), f) for f in range(8)]
        if ref is None:
            want_buf = oracle.pack(lays[0], cols)
            for s in secs:
                oracle.section(lays[0], spec.dtypes, s.op, s.read, s.write, 0, None, want_buf)
            ref = [oracle.unpack(lays[0], want_buf, f) for f in range(8)]
        for f in range(8):
            assert np.array_equal(out[f], ref[f]), (combo, f)


@pytest.mark.parametrize("n", [1000, (1 << 16) + 13])
def test_config3_program_on_several_layouts(ctx, n):
    spec = synth.config3_struct(n)
    cols = synth.record_matrix(3, n, spec.dtypes, spec.elem_bytes)
    secs = synth.random_program(3, spec.n_fields)
    idx = synth.uniform_index(3, 999, n * 16, n)
    eb = spec.elem_bytes
    outs = []
    for O in (oaos(n, eb), osoa(n, eb), OLayout(n, eb, [0] * 32, [64]),
              from_partition(n, eb, [[0, 5, 9], [28, 1, 20], [30, 31]], 1),
              from_partition(n, eb, [[0, 5, 9], [28, 1, 20], [30, 31]], 64)):
        got = _run_sections(ctx, spec, O, secs, cols, idx, "config3")
        outs.append([oracle.unpack(O, got, f) for f in range(spec.n_fields)])
    for o in outs[1:]:
        for f in range(spec.n_fields):
            assert np.array_equal(o[f], outs[0][f])


def test_ops_and_types(ctx):
    n = 3000
    spec = synth.StructSpec(n, [synth.F32, synth.I32, synth.F64, synth.F64, synth.F32, synth.I32, synth.F64],
                            [4, 4, 8, 8, 4, 4, 8])
    cols = synth.record_matrix(11, n, spec.dtypes, spec.elem_bytes)
    secs = [synth.SectionSpec(synth.OP_MULADD3, [0, 1, 2], [3]),
            synth.SectionSpec(synth.OP_SUB2, [2, 3], [6]),
            synth.SectionSpec(synth.OP_SUM, [0, 1, 2, 3], [4]),
            synth.SectionSpec(synth.OP_GEN, [0, 1, 2, 3, 4], [5, 6]),
            synth.SectionSpec(synth.OP_GEN, [0, 6], [0, 6]),      # writes what it reads
            synth.SectionSpec(synth.OP_GEN, [0, 2], [4, 5], 7),
            synth.SectionSpec(synth.OP_GEN, [1, 3, 6], [0], 1)]
    idx = synth.uniform_index(11, 5, n * 7, n)
    eb = spec.elem_bytes
    for O in (oaos(n, eb), osoa(n, eb), OLayout(n, eb, [0, 0, 1, 1, 0, 2, 1], [1, 4, 1])):
        _run_sections(ctx, spec, O, secs, cols, idx, "ops")


@pytest.mark.parametrize("deg", [0, 5])
def test_every_write_type_in_both_write_slots(ctx, deg):
    """Each write type (F32, I32, F64, U32) in each write slot, from the
    direct, per-field gather and span gather kernels: the store of every type
    is checked on its own, integer folds included (bit for bit)."""
    n = 2049
    F32, I32, F64, U32 = synth.F32, synth.I32, synth.F64, synth.U32
    dts = [F32, I32, F64, F32, I32, F64, U32, F32, I32, F64, U32]
    eb = [8 if d == F64 else 4 for d in dts]
    spec = synth.StructSpec(n, dts, eb)
    cols = synth.record_matrix(13, n, dts, eb)
    idx = synth.uniform_index(13, 9, n * max(deg, 1), n)
    secs = [synth.SectionSpec(synth.OP_GEN, [0, 1, 2], [a, b], deg) for a in range(3, 7) for b in range(7, 11)]
    for span in (1, 0):
        ctx.set_option(A.OPT_SPAN_GATHER, span)
        try:
            for O in (oaos(n, eb), osoa(n, eb)):
                _run_sections(ctx, spec, O, secs, cols, idx if deg else None, f"write types span={span}")
        finally:
            ctx.set_option(A.OPT_SPAN_GATHER, 1)


def test_wide_read_sets(ctx):
    n = 4099
    spec = synth.StructSpec(n, [synth.F32] * 30 + [synth.F64] * 4, [4] * 30 + [8] * 4)
    cols = synth.record_matrix(12, n, spec.dtypes, spec.elem_bytes)
    secs = [synth.SectionSpec(synth.OP_GEN, list(range(32)), [32, 33]),
            synth.SectionSpec(synth.OP_GEN, list(range(17)), [30], 3),
            synth.SectionSpec(synth.OP_GEN, list(range(9)), [31, 32], 32)]
    idx = synth.uniform_index(12, 6, n * 32, n)
    _run_sections(ctx, spec, oaos(n, spec.elem_bytes), secs, cols, idx, "wide")


def test_f32_direct_sections_every_read_count_and_layout(ctx):
    """All-F32 direct sections (the straight-line kernel) with 1 to 32 reads
    and one or two writes, on interleaved, single-field and tiled layouts."""
    n = 5 * 1024 + 3
    spec = synth.StructSpec(n, [synth.F32] * 36, [4] * 36)
    cols = synth.record_matrix(14, n, spec.dtypes, spec.elem_bytes)
    secs = [synth.SectionSpec(synth.OP_GEN, [7], [33]),
            synth.SectionSpec(synth.OP_GEN, [0, 3, 5, 8, 13], [34, 35]),
            synth.SectionSpec(synth.OP_GEN, list(range(2, 11)), [32]),
            synth.SectionSpec(synth.OP_SUM, list(range(17)), [33]),
            synth.SectionSpec(synth.OP_GEN, list(range(32)), [34, 35])]
    eb = spec.elem_bytes
    for O in (oaos(n, eb), osoa(n, eb), OLayout(n, eb, [0] * 36, [64]),
              from_partition(n, eb, [list(range(0, 12)), list(range(12, 36))], 8),
              from_partition(n, eb, [[0, 1, 2, 3], [32, 33, 34, 35]], 1)):
        _run_sections(ctx, spec, O, secs, cols, None, "f32 direct")


@pytest.mark.parametrize("group,rd", [
    ([0, 1, 2, 3, 4], [0, 2, 3]),          # 24-byte records (8-byte loads), f64 in the middle
    ([1, 2, 3, 5, 6, 7], [1, 3, 6, 7]),    # 28 bytes (4-byte loads)
    ([0, 1, 3, 4, 5, 6], [0, 1, 3, 5, 6]), # 32 bytes (16-byte loads)
    ([3], [3]),                            # a lone f64 column
])
def test_span_gathers_match_oracle_and_per_field_path(ctx, group, rd):
    n = 3001
    spec = synth.StructSpec(n, [synth.F32, synth.I32, synth.F32, synth.F64, synth.F32, synth.I32,
                                synth.F32, synth.F32, synth.F32, synth.F64],
                            [4, 4, 4, 8, 4, 4, 4, 4, 4, 8])
    cols = synth.record_matrix(21, n, spec.dtypes, spec.elem_bytes)
    wr = [8, 9]
    secs = [synth.SectionSpec(synth.OP_GEN, rd, wr, d) for d in (1, 5, 16, 32)]
    idx = synth.uniform_index(21, 3, n * 32, n)
    O = from_partition(n, spec.elem_bytes, [group] if len(group) > 1 else [], 1)
    got_span = _run_sections(ctx, spec, O, secs, cols, idx, "span")
    ctx.set_option(A.OPT_SPAN_GATHER, 0)
    try:
        got_field = _run_sections(ctx, spec, O, secs, cols, idx, "per-field")
    finally:
        ctx.set_option(A.OPT_SPAN_GATHER, 1)
    assert np.array_equal(got_span, got_field)


def test_gather_out_of_range_indices_are_skipped_and_reported(ctx):
    n = 512
    spec = synth.StructSpec(n, [synth.F32, synth.F32], [4, 4])
    cols = synth.record_matrix(13, n, spec.dtypes, spec.elem_bytes)
    idx = synth.uniform_index(13, 1, n * 2, n)
    idx[5] = n
    idx[17] = -3
    O = osoa(n, spec.elem_bytes)
    st = A.Struct.from_spec(spec)
    L = mirror(st, O)
    buf = dev_bytes(oracle.pack(O, cols))
    want = oracle.pack(O, cols)
    bad = oracle.section(O, spec.dtypes, synth.OP_GEN, [0], [1], 2, idx, want)
    assert bad == 2
    A.section_run(ctx, A.Section(st, A.OP_GEN, [0], [1], 2), L, buf, torch.from_numpy(idx).cuda())
    with pytest.raises(A.AdhaError) as e:
        ctx.check()
    assert e.value.status == A.ERR_INVALID
    ctx.check()  # the flag is cleared
    assert np.array_equal(host(buf, O.nbytes), want)


def test_section_argument_errors(ctx):
    n = 100
    st = A.Struct(n, [A.F32, A.F32])
    L = A.Layout.soa(st)
    sec = A.Section(st, A.OP_GEN, [0], [1], 4)
    buf = torch.zeros(L.nbytes, dtype=torch.uint8, device="cuda")
    idx = torch.zeros(n * 4, dtype=torch.int32, device="cuda")
    with pytest.raises(A.AdhaError):
        A.section_run(ctx, sec, L, buf, None)            # gather without indices
    with pytest.raises(A.AdhaError):
        A.section_run(ctx, sec, L, buf, idx[: n * 2])    # too few indices
    with pytest.raises(A.AdhaError):
        A.section_run(ctx, sec, L, buf[: L.nbytes - 4], idx)
    other = A.Layout.soa(A.Struct(n + 1, [A.F32, A.F32]))
    with pytest.raises(A.AdhaError):
        A.section_run(ctx, sec, other, buf, idx)
    A.section_run(ctx, sec, L, buf, idx)
    ctx.check()
