"""Stencil sections on the GPU against the oracle (which reads the explicit
neighbour array the stencil stands for), on several layouts, through both
gather paths, and the Medical-shaped program at its full size (256^3)."""
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest
import torch

import oracle
from oracle.layout import Layout as OLayout, aos as oaos, soa as osoa, from_partition
from paper_1407_4859_amd import adha as A
from paper_1407_4859_amd import synth
from gpu_util import dev_bytes, fill_aos_device, host, mirror, say

pytestmark = pytest.mark.gpu

OFFS27 = [(dx, dy, dz) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]


@pytest.fixture(scope="module")
def ctx():
    return A.Ctx(0)


def _program(st, grid, extra=True):
    secs = []
    # extra: a 27-point stencil, and a 7-point one over 4 fields with two
    # writes (the multi-record 7-point kernel's widest form)
    more = [([0, 1, 2], [6, 7], OFFS27), ([3, 4, 5, 8], [0, 1], synth.STENCIL7)]
    for rd, wr, offs in synth.medical_sections() + (more if extra else []):
        if offs is None:
            secs.append((A.Section(st, A.OP_GEN, rd, wr, 0), rd, wr, None))
        else:
            secs.append((A.Section.stencil(st, rd, wr, grid, offs), rd, wr, offs))
    return secs


@pytest.mark.parametrize("grid", [(7, 5, 3), (33, 17, 9), (64, 3, 5), (128, 2, 3)])
def test_stencils_match_oracle(ctx, grid):
    """Grids whose rows are a multiple of 64 records take the row-aligned
    kernel forms; the others the general ones."""
    n = grid[0] * grid[1] * grid[2]
    spec = synth.StructSpec(n, [synth.F32] * 9, [4] * 9)
    st = A.Struct.from_spec(spec)
    cols = synth.record_matrix(12, n, spec.dtypes, spec.elem_bytes)
    secs = _program(st, grid)
    for O in (oaos(n, spec.elem_bytes), osoa(n, spec.elem_bytes), OLayout(n, spec.elem_bytes, [0] * 9, [64]),
              from_partition(n, spec.elem_bytes, [[0, 1, 2], [3, 4, 5]], 1),
              from_partition(n, spec.elem_bytes, [[0, 1, 2], [3, 4, 5, 8]], 8)):
        want = oracle.pack(O, cols)
        for _, rd, wr, offs in secs:
            idx = oracle.stencil_index(*grid, offs) if offs else None
            oracle.section(O, spec.dtypes, synth.OP_GEN, rd, wr, len(offs) if offs else 0, idx, want)
        for span in (1, 0):
            ctx.set_option(A.OPT_SPAN_GATHER, span)
            dev = dev_bytes(oracle.pack(O, cols))
            say("stencil", grid, O, "span", span)
            for sec, *_ in secs:
                A.section_run(ctx, sec, mirror(st, O), dev)
            ctx.check()                                   # neighbours off the grid are no error
            assert np.array_equal(host(dev, O.nbytes), want), (grid, O, span)
    ctx.set_option(A.OPT_SPAN_GATHER, 1)


@pytest.mark.parametrize("grid", [(9, 7, 5), (40, 3, 21)])
def test_stencils_with_mixed_types_and_wide_reads(ctx, grid):
    """The generic forms: F64 and I32 fields (typed fold, 8-byte loads),
    5 to 7 read fields (no exact field count), two writes, 27 neighbours."""
    n = grid[0] * grid[1] * grid[2]
    dts = [A.F32, A.F64, A.I32, A.F32, A.F64, A.I32, A.F32, A.F32, A.F64, A.I32]
    eb = [8 if d == A.F64 else 4 for d in dts]
    st = A.Struct(n, dts, eb)
    sdts = [synth.F64 if d == A.F64 else synth.I32 if d == A.I32 else synth.F32 for d in dts]
    cols = synth.record_matrix(21, n, sdts, eb)
    secs = [([0, 3, 6, 7, 2], [9], synth.STENCIL7), ([1, 4, 0], [5, 8], OFFS27),
            ([0, 1, 2, 3, 4, 5, 6], [7], synth.STENCIL7), ([0, 3], [6, 7], OFFS27[:13])]
    secs_h = [(A.Section.stencil(st, rd, wr, grid, offs), rd, wr, offs) for rd, wr, offs in secs]
    for O in (oaos(n, eb), osoa(n, eb), OLayout(n, eb, [0] * 10, [64]),
              from_partition(n, eb, [[0, 3, 6, 7], [1, 4]], 1), from_partition(n, eb, [[0, 1, 2, 3, 4, 5, 6]], 4)):
        want = oracle.pack(O, cols)
        for _, rd, wr, offs in secs_h:
            oracle.section(O, sdts, synth.OP_GEN, rd, wr, len(offs), oracle.stencil_index(*grid, offs), want)
        dev = dev_bytes(oracle.pack(O, cols))
        say("stencil mixed", grid, O)
        for sec, *_ in secs_h:
            A.section_run(ctx, sec, mirror(st, O), dev)
        ctx.check()
        assert np.array_equal(host(dev, O.nbytes), want), (grid, O)


@pytest.mark.parametrize("grid", [(1000, 999, 3), (321, 1023, 7)])
def test_stencil_on_large_irregular_grids(ctx, grid):
    """Millions of records on grids whose sides are not powers of two: the
    kernel's multiply-shift division for the grid coordinates against the
    oracle's neighbour array, every record, on SoA (linear form) and on a
    tiled layout (general form)."""
    n = grid[0] * grid[1] * grid[2]
    spec = synth.StructSpec(n, [synth.F32] * 5, [4] * 5)
    st = A.Struct.from_spec(spec)
    cols = synth.record_matrix(17, n, spec.dtypes, spec.elem_bytes)
    rd, wr = [0, 1, 2], [3]
    idx = oracle.stencil_index(*grid, synth.STENCIL7)
    sec = A.Section.stencil(st, rd, wr, grid, synth.STENCIL7)
    for O in (osoa(n, spec.elem_bytes), OLayout(n, spec.elem_bytes, [0] * 5, [64])):
        want = oracle.pack(O, cols)
        oracle.section(O, spec.dtypes, synth.OP_GEN, rd, wr, 7, idx, want)
        dev = dev_bytes(oracle.pack(O, cols))
        say("stencil large", grid, O)
        A.section_run(ctx, sec, mirror(st, O), dev)
        ctx.check()
        assert np.array_equal(host(dev, O.nbytes), want), (grid, O)


@pytest.mark.timeout(900)
def test_medical_program_full_size(ctx):
    """The Medical-shaped program on a 256^3 image: planned, all-AoS and
    all-SoA runs against the oracle over every record."""
    side = 256
    spec = synth.medical_struct(side)
    n = spec.n
    st = A.Struct.from_spec(spec)
    grid = (side, side, side)
    secs = _program(st, grid, extra=False)
    prog = A.Program(st, [s for s, *_ in secs])
    say("medical full: generating", n, "records on the device")
    src = fill_aos_device(spec, 13)
    want = src.cpu().numpy()
    O = oaos(n, spec.elem_bytes)
    assert O.nbytes == want.size
    cores = max(1, min(16, len(os.sched_getaffinity(0))))
    bounds = [n * i // cores for i in range(cores + 1)]
    for _, rd, wr, offs in secs:
        idx = oracle.stencil_index(*grid, offs) if offs else None
        say("medical full: oracle", rd, wr, "stencil" if offs else "direct")
        with ThreadPoolExecutor(cores) as ex:
            list(ex.map(lambda i: oracle.section(O, spec.dtypes, synth.OP_GEN, rd, wr, len(offs) if offs else 0,
                                                 idx, want, bounds[i], bounds[i + 1]), range(cores)))
    La = A.Layout.aos(st)
    cap = max(La.nbytes, A.Layout.soa(st).nbytes) + (1 << 24)
    buf_a = torch.empty(cap, dtype=torch.uint8, device="cuda")
    buf_b = torch.empty(cap, dtype=torch.uint8, device="cuda")
    back = torch.empty(La.nbytes, dtype=torch.uint8, device="cuda")
    plans = [("planned", A.Plan.create(ctx, prog, A.plan_opts(cost=A.COST_MEASURED, catalogue=A.CAT_FULL, reps=3))),
             ("all-AoS", A.Plan.uniform(prog, La)), ("all-SoA", A.Plan.uniform(prog, A.Layout.soa(st)))]
    for name, plan in plans:
        say("medical full: run", name, plan.choices())
        buf_a[: La.nbytes].copy_(src)
        out_h, in_b = A.run(ctx, plan, La, buf_a, buf_b)
        ctx.check()
        out_l = [L for L in [La] + [plan.candidate(c) for c in range(plan.n_candidates)] if L.h.value == out_h]
        res = buf_b if in_b else buf_a
        if out_l[0].equals(La):
            got = res[: La.nbytes].cpu().numpy()
        else:
            A.remap(ctx, out_l[0], res, La, back)
            ctx.check()
            got = back.cpu().numpy()
        assert np.array_equal(got, want), name
