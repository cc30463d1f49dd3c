"""Sections over narrow (1- and 2-byte) and unsigned typed fields on the GPU
against the oracle: U8, U16, I16 and U32 terms and write fields, and wider
fields that an interleaved group places at offsets that are not multiples of
4 (the byte-wise kernel form).  Results must match bit for bit."""
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest
import torch

import oracle
from oracle import reduce as OR
from oracle.layout import Layout as OLayout, aos as oaos, soa as osoa, from_partition
from paper_1407_4859_amd import adha as A
from paper_1407_4859_amd import synth
from gpu_util import dev_bytes, fill_aos_device, first_diff, host, mirror, say

pytestmark = pytest.mark.gpu

OFFS7 = [(0, 0, 0), (-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0), (0, 0, -1), (0, 0, 1)]


@pytest.fixture(scope="module")
def ctx():
    return A.Ctx(0)


def _layouts(n, eb):
    F = len(eb)
    return (oaos(n, eb), osoa(n, eb), OLayout(n, eb, [0] * F, [64]),
            from_partition(n, eb, [list(range(0, F, 3)), list(range(1, F, 3))], 1),
            from_partition(n, eb, [list(range(0, F, 2))], 8),
            from_partition(n, eb, [[0, 1, 2, 3]], 1))


MIXED_SECTIONS = [synth.SectionSpec(synth.OP_GEN, [0, 1, 2, 3, 4], [8, 9]),
                  synth.SectionSpec(synth.OP_GEN, [0, 3, 5, 6], [7], 6),
                  synth.SectionSpec(synth.OP_GEN, [1, 7, 9], [2, 5]),
                  synth.SectionSpec(synth.OP_MULADD3, [0, 1, 5], [4]),
                  synth.SectionSpec(synth.OP_SUM, [3, 7, 9], [8]),
                  synth.SectionSpec(synth.OP_GEN, [0, 1, 3, 7, 9], [5, 6], 16),
                  synth.SectionSpec(synth.OP_SUB2, [6, 9], [2])]


@pytest.mark.parametrize("n", [1, 255, 4097, 70001])
def test_mixed_narrow_sections_match_oracle(ctx, n):
    spec = synth.mixed_narrow_struct(n)
    st = A.Struct.from_spec(spec)
    cols = synth.record_matrix(31, n, spec.dtypes, spec.elem_bytes)
    idx = synth.uniform_index(31, 7, n * 16, n)
    idx_t = torch.from_numpy(idx).cuda()
    for O in _layouts(n, spec.elem_bytes):
        want = oracle.pack(O, cols)
        dev = dev_bytes(want)
        L = mirror(st, O)
        for s in MIXED_SECTIONS:
            oracle.section(O, spec.dtypes, s.op, s.read, s.write, s.degree, idx if s.degree else None, want)
            say("narrow", n, O, s)
            A.section_run(ctx, A.Section.from_spec(st, s), L, dev, idx_t if s.degree else None)
        ctx.check()
        assert first_diff(host(dev, O.nbytes), want) is None, (O, first_diff(host(dev, O.nbytes), want))


def _medical_program(st, grid):
    out = []
    for rd, wr, offs in synth.medical_sections():
        if offs is None:
            out.append((A.Section(st, A.OP_GEN, rd, wr, 0), rd, wr, None))
        else:
            out.append((A.Section.stencil(st, rd, wr, grid, offs), rd, wr, offs))
    return out


@pytest.mark.parametrize("grid", [(33, 17, 9), (64, 3, 5)])
def test_narrow_medical_stencils_match_oracle(ctx, grid):
    """The Medical-shaped program on the struct with 16-bit intensities, an
    8-bit label and a signed 16-bit field, on small grids and five layouts
    (interleaved trios of 2-byte fields included)."""
    side_n = grid[0] * grid[1] * grid[2]
    spec = synth.medical_narrow_struct(1)
    spec = synth.StructSpec(side_n, spec.dtypes, spec.elem_bytes)
    st = A.Struct.from_spec(spec)
    cols = synth.record_matrix(33, side_n, spec.dtypes, spec.elem_bytes)
    secs = _medical_program(st, grid)
    eb = spec.elem_bytes
    for O in (oaos(side_n, eb), osoa(side_n, eb), from_partition(side_n, eb, [[3, 4, 5]], 1),
              from_partition(side_n, eb, [[0, 1, 2], [6, 7]], 1), from_partition(side_n, eb, [[0, 1, 2, 8]], 64)):
        want = oracle.pack(O, cols)
        dev = dev_bytes(want)
        L = mirror(st, O)
        for sec, rd, wr, offs in secs:
            idx = oracle.stencil_index(*grid, offs) if offs else None
            oracle.section(O, spec.dtypes, synth.OP_GEN, rd, wr, len(offs) if offs else 0, idx, want)
            A.section_run(ctx, sec, L, dev)
        ctx.check()
        assert first_diff(host(dev, O.nbytes), want) is None, (grid, O)


@pytest.mark.timeout(900)
def test_narrow_medical_program_full_size(ctx):
    """The narrow Medical-shaped program on a 256^3 image: the planned
    (measured costs, placed) run and the all-AoS and all-SoA runs against the
    oracle over every record."""
    side = 256
    spec = synth.medical_narrow_struct(side)
    n = spec.n
    st = A.Struct.from_spec(spec)
    grid = (side, side, side)
    secs = _medical_program(st, grid)
    prog = A.Program(st, [s for s, *_ in secs])
    say("narrow medical full: generating", n, "records on the device")
    src = fill_aos_device(spec, 14)
    want = src.cpu().numpy()
    O = oaos(n, spec.elem_bytes)
    assert O.nbytes == want.size
    cores = max(1, min(16, len(os.sched_getaffinity(0))))
    bounds = [n * i // cores for i in range(cores + 1)]
    for _, rd, wr, offs in secs:
        idx = oracle.stencil_index(*grid, offs) if offs else None
        say("narrow medical full: oracle", rd, wr, "stencil" if offs else "direct")
        with ThreadPoolExecutor(cores) as ex:
            list(ex.map(lambda i: oracle.section(O, spec.dtypes, synth.OP_GEN, rd, wr, len(offs) if offs else 0,
                                                 idx, want, bounds[i], bounds[i + 1]), range(cores)))
    La = A.Layout.aos(st)
    back = torch.empty(La.nbytes, dtype=torch.uint8, device="cuda")
    plans = [("planned", A.Plan.create(ctx, prog, A.plan_opts(cost=A.COST_MEASURED, catalogue=A.CAT_FULL, reps=3))),
             ("all-AoS", A.Plan.uniform(prog, La)), ("all-SoA", A.Plan.uniform(prog, A.Layout.soa(st)))]
    arena = torch.empty(max(A.plan_arena(p)[0] for _, p in plans), dtype=torch.uint8, device="cuda")
    for name, plan in plans:
        _, start, end = A.plan_arena(plan)
        say("narrow medical full: run", name, plan.choices())
        A.remap(ctx, La, src, start, arena)
        A.run_placed(ctx, plan, arena)
        A.remap(ctx, end, arena, La, back)
        ctx.check()
        got = back.cpu().numpy()
        assert np.array_equal(got, want), (name, first_diff(got, want))


def test_reduction_type_rules(ctx):
    """U32 columns reduce exactly (zero-extended); narrow read fields are
    refused when the reduction is made, and a 4-byte field a layout leaves
    unaligned when it runs."""
    n = 20_001
    dtypes = [synth.U32, synth.I32, synth.F32, synth.U8, synth.U16]
    eb = [4, 4, 4, 1, 2]
    spec = synth.StructSpec(n, dtypes, eb)
    st = A.Struct.from_spec(spec)
    cols = synth.record_matrix(35, n, dtypes, eb)
    keys = synth.uniform_index(35, 77, n, 3).astype(np.int32)
    cols[1] = keys.view(np.uint8).reshape(n, 4)
    O = osoa(n, eb)
    buf_h = oracle.pack(O, cols)
    out = torch.zeros(3 * 3 * 8, dtype=torch.uint8, device="cuda")
    sec = A.Section.reduce(st, [0, 2], 1, 3, out)
    A.section_run(ctx, sec, mirror(st, O), dev_bytes(buf_h))
    ctx.check()
    table, bad = OR.reduce(O, dtypes, [0, 2], 1, 3, buf_h)
    assert bad == 0
    want = OR.table_cells(table, dtypes, [0, 2])
    got = host(out).view(np.uint64)
    for k in range(3):
        assert got[k * 3] == want[k * 3]                 # U32: exact int64 sum
        assert got[k * 3 + 2] == want[k * 3 + 2]         # count
        assert table[k][0] > 0 and table[k][0] == int(got[k * 3])
    with pytest.raises(A.AdhaError) as e:
        A.Section.reduce(st, [0, 3], 1, 3, out)          # a U8 read field
    assert e.value.status == A.ERR_UNSUPPORTED
    # field 0 (U32) after the U8 and U16 fields in one interleaved group: unaligned
    Ou = OLayout(n, eb, [1, 0, 2, 1, 1], [1, 1, 1])
    assert Ou.S[Ou.group_of[0]] % 4 != 0
    with pytest.raises(A.AdhaError) as e:
        A.section_run(ctx, sec, mirror(st, Ou), dev_bytes(oracle.pack(Ou, cols)))
    assert e.value.status == A.ERR_UNSUPPORTED


# Stencils over every field type: F64 beside 1- and 2-byte reads (the forms
# that load a third dword), narrow reads only (two dwords), 8 reads, and
# F64, I32, F32 and I16 writes; SoA and AoS take linear offsets, the tiled
# and T = 8 layouts do not.  Span option 0 runs the generic fold instead.
MIXED_STENCILS = [([0, 1, 3, 4], [2, 9]), ([3, 7, 9], [8]), ([0, 1, 2, 3, 4, 5, 6, 7], [8, 9]),
                  ([1, 3], [4, 6])]
OFFS_WIDE = OFFS7 + [(1, 1, 0), (-1, 0, 1), (0, -1, -1)]


@pytest.mark.parametrize("grid", [(9, 7, 5), (64, 3, 5)])
@pytest.mark.parametrize("span", [1, 0])
def test_mixed_narrow_stencils_match_oracle(ctx, grid, span):
    n = grid[0] * grid[1] * grid[2]
    spec = synth.mixed_narrow_struct(n)
    st = A.Struct.from_spec(spec)
    cols = synth.record_matrix(37, n, spec.dtypes, spec.elem_bytes)
    ctx.set_option(A.OPT_SPAN_GATHER, span)
    try:
        for O in _layouts(n, spec.elem_bytes):
            want = oracle.pack(O, cols)
            dev = dev_bytes(want)
            L = mirror(st, O)
            for k, (rd, wr) in enumerate(MIXED_STENCILS):
                offs = OFFS7 if k % 2 == 0 else OFFS_WIDE
                idx = oracle.stencil_index(*grid, offs)
                oracle.section(O, spec.dtypes, synth.OP_GEN, rd, wr, len(offs), idx, want)
                say("narrow stencil", grid, span, O, rd, wr)
                A.section_run(ctx, A.Section.stencil(st, rd, wr, grid, offs), L, dev)
            ctx.check()
            assert first_diff(host(dev, O.nbytes), want) is None, (grid, span, O, first_diff(host(dev, O.nbytes), want))
    finally:
        ctx.set_option(A.OPT_SPAN_GATHER, 1)
