"""Stencil sections (CPU only): the oracle's neighbour map pinned by hand,
the host backend against the oracle, validation, and the analytic model."""
import ctypes

import numpy as np
import pytest

import oracle
from oracle import costmodel as OC
from oracle.layout import Layout as OLayout, aos as oaos, soa as osoa, from_partition
from paper_1407_4859_amd import adha as A
from paper_1407_4859_amd import synth


def test_stencil_index_by_hand():
    # a 3 x 2 x 2 grid: r = x + 3*(y + 2*z)
    idx = oracle.stencil_index(3, 2, 2, [(1, 0, 0), (0, -1, 0), (0, 0, 1), (-2, 1, -1)]).reshape(12, 4)
    assert list(idx[0]) == [1, -1, 6, -1]            # (0,0,0): x+1 = 1; y-1 off; z+1 -> 6; x-2 off
    assert list(idx[5]) == [-1, 2, 11, -1]           # (2,1,0): x+1 off; y-1 -> 2; z+1 -> 11; z-1 off
    assert list(idx[11]) == [-1, 8, -1, -1]          # (2,1,1): y-1 -> (2,0,1) = 8; y+1 for (-2,1,-1) off
    assert list(idx[8]) == [-1, -1, -1, 3]           # (2,0,1): (0,1,0) = 3


def _mirror(st, O):
    return A.Layout.create(st, [O.group_of[f] for f in range(len(O.elem_bytes))], [t for _, t in O.groups])


@pytest.mark.parametrize("grid", [(1, 1, 1), (7, 5, 3), (16, 9, 4)])
def test_host_stencils_match_oracle(grid):
    spec = synth.medical_struct(1)
    n = grid[0] * grid[1] * grid[2]
    spec = synth.StructSpec(n, spec.dtypes, spec.elem_bytes)
    st = A.Struct.from_spec(spec)
    cols = synth.record_matrix(11, n, spec.dtypes, spec.elem_bytes)
    offs27 = [(dx, dy, dz) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)]
    for O in (oaos(n, spec.elem_bytes), osoa(n, spec.elem_bytes), OLayout(n, spec.elem_bytes, [0] * 9, [64]),
              from_partition(n, spec.elem_bytes, [[0, 1, 2], [3, 4, 5]], 1)):
        want = oracle.pack(O, cols)
        got = want.copy()
        for rd, wr, offs in synth.medical_sections() + [([0, 1, 2], [6, 7], offs27)]:
            if offs is None:
                sec = A.Section(st, A.OP_GEN, rd, wr, 0)
                oracle.section(O, spec.dtypes, synth.OP_GEN, rd, wr, 0, None, want)
            else:
                sec = A.Section.stencil(st, rd, wr, grid, [o for o in offs if all(abs(v) < g for v, g in zip(o, grid))])
                offs = sec.offsets
                oracle.section(O, spec.dtypes, synth.OP_GEN, rd, wr, len(offs), oracle.stencil_index(*grid, offs), want)
            assert A.host_section_run(sec, _mirror(st, O), got, threads=3) == 0
        assert np.array_equal(got, want), (grid, O)


def test_stencil_validation_and_costs():
    spec = synth.StructSpec(4 * 4 * 4, [synth.F32] * 9, [4] * 9)
    st = A.Struct.from_spec(spec)
    for rd, wr, grid, offs in (([0], [1], (4, 4, 3), [(1, 0, 0)]),        # grid does not hold N
                               ([0], [1], (4, 4, 4), [(4, 0, 0)]),        # offset reaches past the grid
                               ([0], [0], (4, 4, 4), [(1, 0, 0)]),        # writes what it reads
                               ([0], [1], (4, 4, 4), [])):                 # no neighbour
        with pytest.raises(A.AdhaError):
            A.Section.stencil(st, rd, wr, grid, offs)
    s = A.Section.stencil(st, [0, 1], [2], (4, 4, 4), synth.STENCIL7)
    assert s.bytes == 64 * (8 + 4)                     # every element once, no index bytes
    prog = A.Program(st, [s])
    opts = A.plan_opts(cost=A.COST_ANALYTIC, cap_bytes=64)
    h = ctypes.c_void_p()
    A.check(A.lib().adha_plan_create(None, prog.h, ctypes.byref(opts), None, 0, None, ctypes.byref(h)))
    pl = A.Plan(h, 1)
    T, _ = pl.tables()
    for c in range(pl.n_candidates):
        gof, tiles = pl.candidate(c).groups(9)
        O = OLayout(64, spec.elem_bytes, gof, tiles)
        # a stencil is priced as a direct pass over its fields
        assert T[0][c] == pytest.approx(OC.section_us([0, 1], [2], 0, O), rel=1e-12)
