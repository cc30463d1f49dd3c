"""Host-side checks of the C-ABI library (no device work): it loads, exports
every declared symbol, and its host logic (layout address map, affinity,
greedy clustering, shortest path, features) agrees with the oracle."""
import ctypes
import random
import subprocess

import numpy as np
import pytest

from oracle import costmodel as OC
from oracle import planner as OP
from oracle.layout import Layout as OLayout, aos as oaos, soa as osoa
from paper_1407_4859_amd import adha as A
from paper_1407_4859_amd import synth


def test_library_exports_every_declared_symbol():
    out = subprocess.run(["nm", "-D", "--defined-only", A.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = {ln.split()[-1] for ln in out.splitlines() if " T " in ln}
    declared = A.header_symbols()
    assert len(declared) >= 45
    missing = [s for s in declared if s not in exported]
    assert not missing, missing
    lib = A.lib()
    for s in declared:
        assert hasattr(lib, s)
    assert set(A._SIGS) == set(declared)


def test_status_strings_and_version():
    lib = A.lib()
    assert lib.adha_status_string(0) == b"ok"
    assert lib.adha_status_string(-1) == b"invalid argument"
    assert lib.adha_version() >= 10000


def _rand_layout(rng, st, eb):
    F = len(eb)
    ng = rng.randint(1, F)
    gof = [rng.randrange(ng) for _ in range(F)]
    used = {g: i for i, g in enumerate(sorted(set(gof)))}
    gof = [used[g] for g in gof]
    tiles = [rng.choice([1, 2, 8, 64, 256]) for _ in used]
    return gof, tiles


def test_layout_address_map_matches_oracle():
    rng = random.Random(3)
    for trial in range(40):
        F = rng.randint(1, 12)
        eb = [rng.choice([1, 2, 4, 8]) for _ in range(F)]
        dts = [A.RAW] * F
        n = rng.choice([0, 1, 63, 64, 65, 1000, 1 << 20])
        st = A.Struct(n, dts, eb)
        gof, tiles = _rand_layout(rng, st, eb)
        L = A.Layout.create(st, gof, tiles)
        O = OLayout(n, eb, gof, tiles)
        assert L.nbytes == O.nbytes
        g_lib, t_lib = L.groups(F)
        assert [O.group_of[f] for f in range(F)] == g_lib
        assert [t for _, t in O.groups] == t_lib
        for r in sorted({r for r in (0, 1, n // 2, n - 1) if 0 <= r < n}):
            for f in range(F):
                assert L.addr(r, f) == O.addr(r, f)
    st = A.Struct(10, [A.F32] * 3)
    assert A.Layout.aos(st).nbytes == oaos(10, [4] * 3).nbytes
    assert A.Layout.soa(st).nbytes == osoa(10, [4] * 3).nbytes
    assert A.Layout.create(st, [1, 0, 1], [1, 1]).equals(A.Layout.create(st, [0, 1, 0], [1, 1]))
    assert not A.Layout.aos(st).equals(A.Layout.soa(st))


def test_remap_launch_description_covers_every_byte():
    """The host side of a remap launch: tiles of R records (a multiple of 64
    and of every tile), LDS within 64 KiB, and the main kernel's tiles plus
    the tail kernel's bytes cover the destination exactly."""
    rng = random.Random(8)
    for trial in range(300):
        F = rng.randint(1, 24)
        eb = [rng.choice([1, 2, 4, 8] if trial % 4 == 3 else [4, 8]) for _ in range(F)]
        n = rng.choice([0, 1, 63, 64, 65, 4095, 100003, 1 << 22, (1 << 26) + 5])
        st = A.Struct(n, [A.RAW] * F, eb)
        la, lb = (A.Layout.create(st, *_rand_layout(rng, st, eb)) for _ in range(2))
        info = A.describe(la, lb, 256)
        O = OLayout(n, eb, *lb.groups(F))
        R = info["tile_records"]
        S = sum(eb)
        if R:
            tmax = max(max(la.groups(F)[1]), max(lb.groups(F)[1]))
            assert R % max(64, tmax) == 0 and R * S <= 256 * info["slots"] * 16
            assert info["lds_bytes"] <= 65536 and info["full_tiles"] == n // R
            # 1- and 2-byte fields take the byte mode of the same tile kernel
            assert info["byte_path"] == (0 if all(e in (4, 8) for e in eb) else 1) or n < R
        else:
            assert info["full_tiles"] == 0
        assert info["full_tiles"] * R * S + info["tail_bytes"] == O.nbytes or n == 0
        if info["full_tiles"]:
            assert 1 <= info["grid"] <= 256 * info["wg_per_cu"]


def test_invalid_host_arguments_are_rejected():
    with pytest.raises(A.AdhaError) as e:
        A.Struct(-1, [A.F32])
    assert e.value.status == A.ERR_INVALID
    for dt, eb in ((A.F32, 8), (A.F64, 4), (A.I32, 2), (A.RAW, 3), (7, 4)):
        with pytest.raises(A.AdhaError):
            A.Struct(10, [dt], [eb])
    st = A.Struct(10, [A.F32, A.F32, A.F64, A.RAW], [4, 4, 8, 2])
    for gof, tiles in (([0, 0, 0, 0], [3]), ([0, 0, 0, 0], [512]), ([0, 1, 0, 0], [1]),
                       ([0, 2, 2, 2], [1, 1, 1]), ([0, 0, 0, 9], [1])):
        with pytest.raises(A.AdhaError) as e:
            A.Layout.create(st, gof, tiles)
        assert e.value.status == A.ERR_INVALID
    bad_sections = [
        (A.OP_GEN, [], [1], 0), (A.OP_GEN, [0], [], 0), (A.OP_GEN, [0, 0], [1], 0),
        (A.OP_GEN, [0], [9], 0), (A.OP_GEN, [0, 1], [1], 4),        # gather writes what it reads
        (A.OP_GEN, [0], [1], 33), (A.OP_MULADD3, [0, 1], [2], 0), (A.OP_SUB2, [0, 1], [2], 2),
        (A.OP_GEN, [3], [0], 0),                                     # RAW field in a section
        (A.OP_SUM, [0, 1], [2, 1], 0), (9, [0], [1], 0)]
    for op, rd, wr, d in bad_sections:
        with pytest.raises(A.AdhaError):
            A.Section(st, op, rd, wr, d)
    with pytest.raises(A.AdhaError):
        A.Section(A.Struct(4, [A.I32, A.I32]), A.OP_SUM, [0], [1])  # SUM needs an fp write
    s = A.Section(st, A.OP_GEN, [0, 2], [1], 16)
    assert s.bytes == 10 * (4 * 16 + 16 * 12 + 4)
    # a stencil's algorithmic bytes count every element once (neighbours
    # are records of the same arrays), like a direct pass
    grid_st = A.Struct(2 * 5 * 1, [A.F32, A.F32, A.F64])
    sten = A.Section.stencil(grid_st, [0, 2], [1], (2, 5, 1), [(0, 0, 0), (1, 0, 0), (0, -1, 0)])
    assert sten.bytes == 10 * (4 + 8 + 4)
    with pytest.raises(A.AdhaError):
        A.Layout.aos(st).addr(10, 0)


def _prog(st_spec, secs):
    st = A.Struct.from_spec(st_spec)
    ss = [A.Section.from_spec(st, s) for s in secs]
    return st, ss, A.Program(st, ss)


def test_affinity_and_ods_match_oracle():
    rng = random.Random(4)
    spec = synth.config3_struct(1000)
    for seed in range(1, 9):
        secs = synth.random_program(seed, spec.n_fields)
        st, ss, prog = _prog(spec, secs)
        osecs = [(s.read, s.write, s.degree) for s in secs]
        for _ in range(6):
            i = rng.randrange(len(secs))
            j = rng.randrange(i, len(secs))
            assert prog.affinity(i, j) == OP.affinity(osecs[i:j + 1], spec.n_fields)
            cap = rng.choice([16, 24, 32, 64, 128])
            parts = OP.ods_greedy(osecs[i:j + 1], spec.elem_bytes, cap)
            for tile in (1, 64):
                L = prog.ods(i, j, cap, tile)
                O = OP.from_partition(spec.n, spec.elem_bytes, parts, tile)
                gof, tiles = L.groups(spec.n_fields)
                assert gof == [O.group_of[f] for f in range(spec.n_fields)]
                assert tiles == [t for _, t in O.groups]


def test_table3_split_through_the_library():
    spec = synth.StructSpec(100, [synth.F32] * 32, [4] * 32)
    st, ss, prog = _prog(spec, [synth.SectionSpec(synth.OP_GEN, list(range(31)), [31])])
    L = prog.ods(0, 0, 32, 1)
    gof, tiles = L.groups(32)
    assert gof == [f // 8 for f in range(32)] and tiles == [1, 1, 1, 1]


def test_pdl_solve_matches_oracle_and_bruteforce():
    rng = random.Random(6)
    for _ in range(150):
        k, C = rng.randint(1, 5), rng.randint(1, 6)
        T = [[float(rng.randint(0, 40)) for _ in range(C)] for _ in range(k)]
        R = [[0.0 if a == b else float(rng.randint(0, 40)) for b in range(C)] for a in range(C)]
        R0 = [float(rng.randint(0, 40)) for _ in range(C)]
        for r0 in (None, R0):
            cost, path = A.pdl_solve(T, R, r0)
            ocost, opath = OP.pdl_dp(T, R, r0)
            assert cost == ocost and path == opath
            if C ** k <= 4000:
                assert cost == OP.pdl_bruteforce(T, R, r0)[0]


def test_analytic_plan_catalogue_matches_oracle():
    spec = synth.config3_struct(1 << 12)
    secs = synth.random_program(3, spec.n_fields)
    st, ss, prog = _prog(spec, secs)
    opts = A.plan_opts(cost=A.COST_ANALYTIC, cap_bytes=64)
    pl = A.Plan(ctypes.c_void_p(), len(secs))
    h = ctypes.c_void_p()
    A.check(A.lib().adha_plan_create(None, prog.h, ctypes.byref(opts), None, 0, None, ctypes.byref(h)))
    pl.h = h
    osecs = [(s.read, s.write, s.degree) for s in secs]
    cat = OP.catalogue(osecs, spec.n, spec.elem_bytes, 64, full=True)
    assert pl.n_candidates == len(cat)
    for c, O in enumerate(cat):
        gof, tiles = pl.candidate(c).groups(spec.n_fields)
        assert gof == [O.group_of[f] for f in range(spec.n_fields)]
        assert tiles == [t for _, t in O.groups]
    T, R = pl.tables()
    cost, path = OP.pdl_dp(T, R)
    assert pl.choices() == path
    assert abs(pl.cost - cost) <= 1e-9 * cost


class _FakeDev:
    """Stands in for a device tensor at creation time (nothing is read or
    written through it until a run)."""

    def __init__(self, addr, nbytes):
        self.addr, self.nbytes = addr, nbytes

    def data_ptr(self):
        return self.addr

    def numel(self):
        return self.nbytes

    def element_size(self):
        return 1


def test_reduction_sections_validate_and_plan_like_the_oracle():
    spec = synth.StructSpec(1 << 12, [synth.F32] * 6 + [synth.I32, synth.F64], [4] * 7 + [8])
    st = A.Struct.from_spec(spec)
    out = _FakeDev(1 << 20, 5 * 4 * 8)
    r = A.Section.reduce(st, [0, 2, 7], 6, 5, out)
    assert r.bytes == spec.n * (4 + 4 + 8 + 4)
    bad = [([0], 2, 5, out),                                   # key is F32
           ([0, 6], 6, 5, out),                                # key also read
           ([0], -1, 3, out),                                  # no key, several rows
           ([0], 6, 0, out),                                   # no rows
           ([0, 1, 2], 6, 5, _FakeDev(1 << 20, 5 * 4 * 8 - 1)),  # table does not fit
           ([0], 6, 5, _FakeDev((1 << 20) + 8, 4096)),         # misaligned
           ([0] * 2, 6, 5, out),                               # field twice
           (list(range(6)), 6, 4096 // 7 + 1, _FakeDev(1 << 20, 1 << 20))]   # too many cells
    for rd, key, nk, o in bad:
        with pytest.raises(A.AdhaError) as e:
            A.Section.reduce(st, rd, key, nk, o)
        assert e.value.status == A.ERR_INVALID
    with pytest.raises(A.AdhaError):
        A.Section(st, A.OP_REDUCE, [0], [1], 0)             # not through adha_section_create
    # a program with a reduction: affinity, catalogue and analytic tables as
    # the oracle's with the key taken as one more streamed read
    g = A.Section(st, A.OP_GEN, [0, 1, 3], [4], 0)
    prog = A.Program(st, [g, r])
    osecs = [([0, 1, 3], [4], 0), ([0, 2, 6, 7], [], 0)]
    assert prog.affinity(0, 1) == OP.affinity(osecs, spec.n_fields)
    opts = A.plan_opts(cost=A.COST_ANALYTIC, cap_bytes=64)
    h = ctypes.c_void_p()
    A.check(A.lib().adha_plan_create(None, prog.h, ctypes.byref(opts), None, 0, None, ctypes.byref(h)))
    pl = A.Plan(h, 2)
    cat = OP.catalogue(osecs, spec.n, spec.elem_bytes, 64)
    assert pl.n_candidates == len(cat)
    T, _ = pl.tables()
    for c, O in enumerate(cat):
        for s, (rd, wr, d) in enumerate(osecs):
            assert T[s][c] == pytest.approx(OC.section_us(rd, wr, d, O), rel=1e-12)


def test_analytic_plans_over_both_devices():
    """Node graph of a plan over the GPU and the host: section costs per
    device, moves between devices cost a transfer (plus the GPU remap when
    the layout changes); the chosen path is the shortest over those nodes."""
    for n in (1 << 8, 1 << 20):
        spec = synth.config3_struct(n)
        secs = synth.random_program(5, spec.n_fields)
        st, ss, prog = _prog(spec, secs)
        for init in (A.INIT_FREE, A.INIT_HOST_AOS):
            opts = A.plan_opts(cost=A.COST_ANALYTIC, cap_bytes=64, devices=A.DEVICES_GPU_HOST, init=init)
            h = ctypes.c_void_p()
            A.check(A.lib().adha_plan_create(None, prog.h, ctypes.byref(opts), None, 0, None, ctypes.byref(h)))
            pl = A.Plan(h, len(secs))
            C = pl.n_candidates
            T, R = pl.node_tables()
            assert len(T[0]) == 2 * C and len(R) == 2 * C
            Tg, Rg = pl.tables()
            S = spec.record_bytes * n
            xfer = 10.0 + S / 5.0e4
            rem_h = 30.0 + 2.0 * S / 4.0e4
            for s in range(len(secs)):
                assert T[s][:C] == Tg[s]
                for c in range(0, C, 7):
                    want = 30.0 + OC.bytes_per_record(secs[s].read, secs[s].write, secs[s].degree,
                                                      OP.catalogue([(x.read, x.write, x.degree) for x in secs],
                                                                   n, spec.elem_bytes, 64)[c]) * n / 4.0e4
                    assert T[s][C + c] == pytest.approx(want, rel=1e-12)
            for a in range(0, 2 * C, 5):
                for b in range(0, 2 * C, 3):
                    if a == b:
                        continue
                    la, lb, ga, gb = a % C, b % C, a < C, b < C
                    if ga and gb:
                        want = Rg[la][lb]
                    elif not ga and not gb:
                        want = 0.0 if la == lb else rem_h
                    else:
                        want = xfer + (0.0 if la == lb else Rg[0][1])
                    assert R[a][b] == pytest.approx(want, rel=1e-12)
            R0 = None
            if init == A.INIT_HOST_AOS:
                R0 = [0.0 if m == C else R[C][m] for m in range(2 * C)]
            cost, path = OP.pdl_dp(T, R, R0)
            assert [m % C for m in path] == pl.choices()
            assert [int(m >= C) for m in path] == pl.devices()
            assert pl.cost == pytest.approx(cost, rel=1e-12)
        if n == 1 << 20:
            assert pl.devices() == [0] * len(secs)       # a large struct stays on the GPU
    with pytest.raises(A.AdhaError):
        opts = A.plan_opts(cost=A.COST_ANALYTIC, init=A.INIT_HOST_AOS)   # host start needs both devices
        h = ctypes.c_void_p()
        A.check(A.lib().adha_plan_create(None, prog.h, ctypes.byref(opts), None, 0, None, ctypes.byref(h)))


# ---------------------------------------------------------------- placed layouts
def test_placed_layouts_match_oracle_and_reject_bad_bases():
    rng = random.Random(17)
    for trial in range(25):
        F = rng.randint(1, 9)
        eb = [rng.choice([1, 2, 4, 8]) for _ in range(F)]
        n = rng.choice([1, 63, 64, 1000])
        st = A.Struct(n, [A.RAW] * F, eb)
        gof, tiles = _rand_layout(rng, st, eb)
        L = A.Layout.create(st, gof, tiles)
        O = OLayout(n, eb, gof, tiles)
        # the groups in shuffled order, each at a 256-aligned slot with a gap
        order = list(range(len(O.groups)))
        rng.shuffle(order)
        at, bases = 256 * rng.randint(0, 3), [0] * len(O.groups)
        for g in order:
            bases[g] = at
            at += -(-O.B[g] // 256) * 256 + 256 * rng.randint(0, 2)
        P, OP_ = L.place(bases), O.placed(bases)
        assert P.bases() == bases and P.nbytes == OP_.nbytes
        for f in range(F):
            for r in {0, n - 1, n // 2}:
                assert P.addr(r, f) == OP_.addr(r, f)
        assert not P.equals(L) or bases == O.base
    st = A.Struct(1000, [A.F32] * 3)
    L = A.Layout.soa(st)
    for bad in ([0, 4096, 4100], [0, 4096], [0, 0, 8192], [0, 3840, 8192]):   # misaligned, count, overlaps
        with pytest.raises(A.AdhaError):
            L.place(bad)
    assert L.place([8192, 0, 4096]).nbytes == 8192 + 4096


def test_pdl_prefers_the_cheaper_remap_when_sections_cost_the_same():
    """Two candidates that price every section alike and differ only in what
    a remap into them moves: the shortest path takes the one that keeps more
    groups in place, as brute force over every assignment does."""
    n, eb = 1 << 16, [4] * 6
    L0 = OLayout(n, eb, [0, 0, 0, 1, 2, 3], [1, 1, 1, 1])      # {0,1,2} interleaved
    L1 = OLayout(n, eb, [0, 0, 0, 1, 1, 2], [1, 1, 1])         # keeps {0,1,2}, joins {3,4}
    L2 = OLayout(n, eb, [0, 1, 1, 2, 2, 3], [1, 1, 1, 1])      # breaks {0,1,2} up
    cands = [L0, L1, L2]
    R = [[OC.remap_us(a, b) for b in cands] for a in cands]
    assert R[0][1] < R[0][2]
    T = [[1.0, 50.0, 50.0], [90.0, 10.0, 10.0]]
    cost, path = OP.pdl_dp(T, R)
    bf_cost, bf_path = OP.pdl_bruteforce(T, R)
    assert path == bf_path == [0, 1] and cost == pytest.approx(bf_cost)
    lib_path = (ctypes.c_uint32 * 2)()
    c = ctypes.c_double()
    flat = lambda m: (ctypes.c_double * (len(m) * len(m[0])))(*[v for row in m for v in row])
    A.check(A.lib().adha_pdl_solve(2, 3, flat(T), flat(R), None, lib_path, ctypes.byref(c)))
    assert list(lib_path) == [0, 1] and c.value == pytest.approx(cost)


def test_analytic_plan_placement_keeps_shared_groups_in_place():
    """The placed sequence of analytic plans of random programs: a group two
    consecutive layouts share keeps its base, a new group never overlaps a
    group of the layout before it, everything fits the arena, and the
    remap cost of every pair is that of its moving fields."""
    spec = synth.config3_struct(1 << 16)
    st = A.Struct.from_spec(spec)
    for seed in (3, 11, 12, 13):
        secs = synth.random_program(seed, spec.n_fields)
        prog = A.Program(st, [A.Section.from_spec(st, s) for s in secs])
        opts = A.plan_opts(cost=A.COST_ANALYTIC, cap_bytes=64)
        h = ctypes.c_void_p()
        A.check(A.lib().adha_plan_create(None, prog.h, ctypes.byref(opts), None, 0, None, ctypes.byref(h)))
        pl = A.Plan(h, len(secs))
        arena, start, end = A.plan_arena(pl)
        placed = [A.plan_placed(pl, i) for i in range(len(secs) + 1)]
        assert start.equals(placed[0]) and end.equals(placed[-1])
        assert start.equals(pl.candidate(pl.choices()[0]))          # canonical, at offset 0
        for i in range(len(secs) + 1):
            gof, tiles = placed[i].groups(spec.n_fields)
            O = OLayout(spec.n, spec.elem_bytes, gof, tiles).placed(placed[i].bases())
            assert O.nbytes <= arena
            if i == 0:
                prev = O
                continue
            for g, grp in enumerate(O.groups):
                if grp in prev.groups:
                    assert O.base[g] == prev.base[prev.groups.index(grp)]
                else:
                    a, b = O.region(g)
                    for h2 in range(len(prev.groups)):
                        c2, d2 = prev.region(h2)
                        assert b <= c2 or d2 <= a
            prev = O
