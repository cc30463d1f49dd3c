"""GPU tests of planning with measured costs and of plan execution: the
program run under any plan equals the oracle's program; the shortest path
over the measured tables equals brute-force enumeration."""
import numpy as np
import pytest
import torch

import oracle
from oracle import planner as OP
from oracle.layout import Layout as OLayout, aos as oaos
from paper_1407_4859_amd import adha as A
from paper_1407_4859_amd import synth
from gpu_util import dev_bytes, host, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    return A.Ctx(0)


def _oracle_program(spec, secs, cols, idx):
    L = oaos(spec.n, spec.elem_bytes)
    buf = oracle.pack(L, cols)
    for s in secs:
        oracle.section(L, spec.dtypes, s.op, s.read, s.write, s.degree, idx, buf)
    return [oracle.unpack(L, buf, f) for f in range(spec.n_fields)]


def _olayout(spec, lay: A.Layout):
    gof, tiles = lay.groups(spec.n_fields)
    return OLayout(spec.n, spec.elem_bytes, gof, tiles)


def _run_and_read(ctx, spec, plan, cols, idx_t):
    """Start from the plan's first layout, run, return per-field bytes."""
    first = plan.candidate(plan.choices()[0])
    O1 = _olayout(spec, first)
    cap = max(plan.candidate(c).nbytes for c in range(plan.n_candidates)) + 256
    a = dev_bytes(oracle.pack(O1, cols), extra=cap - O1.nbytes)
    b = torch.empty(cap, dtype=torch.uint8, device="cuda")
    out_h, in_b = A.run(ctx, plan, first, a, b, idx_t)
    ctx.check()
    final = None
    for c in range(plan.n_candidates):
        if plan.candidate(c).h.value == out_h:
            final = plan.candidate(c)
    assert final is not None
    Of = _olayout(spec, final)
    buf = host(b if in_b else a, Of.nbytes)
    return [oracle.unpack(Of, buf, f) for f in range(spec.n_fields)]


def test_config1_measured_plan(ctx):
    n = 65536
    spec = synth.config1_struct(n)
    st = A.Struct.from_spec(spec)
    secs = synth.config1_sections()
    prog = A.Program(st, [A.Section.from_spec(st, s) for s in secs])
    plan = A.Plan.create(ctx, prog, A.plan_opts(cost=A.COST_MEASURED, catalogue=A.CAT_AOS_SOA, reps=5))
    assert plan.n_candidates == 2
    T, R = plan.tables()
    say("config1 tables", T, R, "choice", plan.choices())
    bcost, bpath = OP.pdl_bruteforce(T, R)
    assert abs(plan.cost - bcost) <= 1e-9 * bcost
    assert OP.path_cost(T, R, plan.choices()) == pytest.approx(bcost, rel=1e-12)
    cols = synth.record_matrix(1, n, spec.dtypes, spec.elem_bytes)
    want = _oracle_program(spec, secs, cols, None)
    got = _run_and_read(ctx, spec, plan, cols, None)
    for f in range(8):
        assert np.array_equal(got[f], want[f]), f


@pytest.mark.parametrize("cost", [A.COST_MEASURED, A.COST_ANALYTIC])
def test_config3_plan_runs_to_the_oracle_result(ctx, cost):
    n = (1 << 16) + 5
    spec = synth.config3_struct(n)
    st = A.Struct.from_spec(spec)
    secs = synth.random_program(3, spec.n_fields)
    prog = A.Program(st, [A.Section.from_spec(st, s) for s in secs])
    idx = synth.uniform_index(3, 999, n * 16, n)
    idx_t = torch.from_numpy(idx).cuda()
    plan = A.Plan.create(ctx, prog, A.plan_opts(cost=cost, catalogue=A.CAT_FULL, cap_bytes=64, reps=3),
                         idx=idx_t)
    say("config3 plan", plan.choices(), "candidates", plan.n_candidates, "cost us", plan.cost)
    T, R = plan.tables()
    cost_dp, path = OP.pdl_dp(T, R)
    assert path == plan.choices() and cost_dp == pytest.approx(plan.cost, rel=1e-12)
    cols = synth.record_matrix(3, n, spec.dtypes, spec.elem_bytes)
    want = _oracle_program(spec, secs, cols, idx)
    got = _run_and_read(ctx, spec, plan, cols, idx_t)
    for f in range(spec.n_fields):
        assert np.array_equal(got[f], want[f]), f
    for lay in (A.Layout.aos(st), A.Layout.soa(st)):
        got = _run_and_read(ctx, spec, A.Plan.uniform(prog, lay), cols, idx_t)
        for f in range(spec.n_fields):
            assert np.array_equal(got[f], want[f]), f


def test_run_rejects_small_buffers_and_starts_from_any_layout(ctx):
    n = 4096
    spec = synth.config3_struct(n)
    st = A.Struct.from_spec(spec)
    secs = synth.random_program(5, spec.n_fields)
    prog = A.Program(st, [A.Section.from_spec(st, s) for s in secs])
    idx = synth.uniform_index(5, 999, n * 16, n)
    idx_t = torch.from_numpy(idx).cuda()
    plan = A.Plan.create(ctx, prog, A.plan_opts(cost=A.COST_ANALYTIC))
    small = torch.empty(1024, dtype=torch.uint8, device="cuda")
    with pytest.raises(A.AdhaError):
        A.run(ctx, plan, A.Layout.aos(st), small, small, idx_t)
    # start in SoA: the run remaps into the first planned layout first
    cols = synth.record_matrix(5, n, spec.dtypes, spec.elem_bytes)
    from oracle.layout import soa as osoa
    Os = osoa(n, spec.elem_bytes)
    cap = max(plan.candidate(c).nbytes for c in range(plan.n_candidates)) + Os.nbytes
    a = dev_bytes(oracle.pack(Os, cols), extra=cap - Os.nbytes)
    b = torch.empty(cap, dtype=torch.uint8, device="cuda")
    out_h, in_b = A.run(ctx, plan, A.Layout.soa(st), a, b, idx_t)
    ctx.check()
    final = [plan.candidate(c) for c in range(plan.n_candidates) if plan.candidate(c).h.value == out_h][0]
    Of = _olayout(spec, final)
    buf = host(b if in_b else a, Of.nbytes)
    want = _oracle_program(spec, secs, cols, idx)
    for f in range(spec.n_fields):
        assert np.array_equal(oracle.unpack(Of, buf, f), want[f])


def _olayout_placed(spec, lay: A.Layout):
    return _olayout(spec, lay).placed(lay.bases())


def _run_placed_and_read(ctx, spec, plan, cols, idx_t):
    """The plan in one arena (adha_run_placed): the data starts in the plan's
    start layout; returns per-field bytes read through the end layout."""
    arena_bytes, start, end = A.plan_arena(plan)
    Os = _olayout(spec, start)
    assert start.bases() == Os.base                     # canonical, from the arena's start
    arena = dev_bytes(oracle.pack(Os, cols), extra=arena_bytes - Os.nbytes + 256, fill=0x3C)
    A.run_placed(ctx, plan, arena, idx_t)
    ctx.check()
    Oe = _olayout_placed(spec, end)
    buf = host(arena)
    return [oracle.unpack(Oe, buf, f) for f in range(spec.n_fields)]


@pytest.mark.parametrize("cost", [A.COST_MEASURED, A.COST_ANALYTIC])
def test_config3_placed_run_matches_the_oracle(ctx, cost):
    """Plans priced for in-place remaps, run in one arena: the program's
    result equals the oracle's whatever the plan, and the measured remap
    table varies with the fields each pair moves."""
    n = (1 << 16) + 5
    spec = synth.config3_struct(n)
    st = A.Struct.from_spec(spec)
    secs = synth.random_program(3, spec.n_fields)
    prog = A.Program(st, [A.Section.from_spec(st, s) for s in secs])
    idx = synth.uniform_index(3, 999, n * 16, n)
    idx_t = torch.from_numpy(idx).cuda()
    plan = A.Plan.create(ctx, prog, A.plan_opts(cost=cost, catalogue=A.CAT_FULL, cap_bytes=64, reps=3),
                         idx=idx_t)
    T, R = plan.tables()
    cost_dp, path = OP.pdl_dp(T, R)
    assert path == plan.choices() and cost_dp == pytest.approx(plan.cost, rel=1e-12)
    want = _oracle_program(spec, secs, synth.record_matrix(3, n, spec.dtypes, spec.elem_bytes), idx)
    cols = synth.record_matrix(3, n, spec.dtypes, spec.elem_bytes)
    say("placed run", plan.choices(), "arena", A.plan_arena(plan)[0])
    got = _run_placed_and_read(ctx, spec, plan, cols, idx_t)
    for f in range(spec.n_fields):
        assert np.array_equal(got[f], want[f]), f
    for lay in (A.Layout.aos(st), A.Layout.soa(st)):
        got = _run_placed_and_read(ctx, spec, A.Plan.uniform(prog, lay), cols, idx_t)
        for f in range(spec.n_fields):
            assert np.array_equal(got[f], want[f]), f
    # remap costs depend on the pair: against the bytes each pair moves
    C = plan.n_candidates
    cands = [_olayout(spec, plan.candidate(c)) for c in range(C)]
    mb = np.array([[OP.remap_bytes(cands[a], cands[b]) for b in range(C)] for a in range(C)], float)
    Rm = np.array(R)
    off = ~np.eye(C, dtype=bool)
    assert len(np.unique(np.round(Rm[off], 6))) > 5            # not one figure for every pair
    assert np.all(Rm[mb == 0] == 0)
    if cost == A.COST_ANALYTIC:
        from oracle import costmodel as OC
        for a in range(C):
            for b in range(C):
                assert R[a][b] == pytest.approx(OC.remap_us(cands[a], cands[b]), rel=1e-12)


def test_measured_remap_costs_follow_the_moving_bytes(ctx):
    """At 2^22 records (600 MB per layout) the measured in-place remap of
    every ordered pair of the catalogue: pairs that move more bytes take
    longer, and pairs that move a quarter of the struct or less are well
    below the whole-struct AoS -> SoA remap."""
    n = 1 << 22
    spec = synth.config3_struct(n)
    st = A.Struct.from_spec(spec)
    secs = synth.random_program(3, spec.n_fields)
    prog = A.Program(st, [A.Section.from_spec(st, s) for s in secs])
    idx_t = synth.uniform_index_torch(3, 999, n * 16, n, "cuda")
    plan = A.Plan.create(ctx, prog, A.plan_opts(cost=A.COST_MEASURED, catalogue=A.CAT_FULL, cap_bytes=64, reps=3),
                         idx=idx_t)
    T, R = plan.tables()
    C = plan.n_candidates
    cands = [_olayout(spec, plan.candidate(c)) for c in range(C)]
    mb = np.array([[OP.remap_bytes(cands[a], cands[b]) for b in range(C)] for a in range(C)], float)
    Rm = np.array(R)
    sel = ~np.eye(C, dtype=bool) & (mb > 0)
    r = np.corrcoef(mb[sel], Rm[sel])[0, 1]
    whole = Rm[0][1]                                           # AoS -> SoA moves every field
    small = Rm[sel & (mb <= mb.max() / 4)]
    say("remap pairs", int(sel.sum()), "corr", r, "whole us", whole, "median small us", np.median(small))
    assert r > 0.8
    assert np.median(small) < 0.5 * whole


def test_placed_run_from_aos_init(ctx):
    """INIT_AOS: the start layout is AoS and the entry remap is part of the
    placed run."""
    n = 20_003
    spec = synth.config3_struct(n)
    st = A.Struct.from_spec(spec)
    secs = synth.random_program(7, spec.n_fields)
    prog = A.Program(st, [A.Section.from_spec(st, s) for s in secs])
    idx = synth.uniform_index(7, 999, n * 16, n)
    idx_t = torch.from_numpy(idx).cuda()
    plan = A.Plan.create(ctx, prog, A.plan_opts(cost=A.COST_ANALYTIC, init=A.INIT_AOS), idx=idx_t)
    _, start, _ = A.plan_arena(plan)
    assert start.equals(A.Layout.aos(st))
    cols = synth.record_matrix(7, n, spec.dtypes, spec.elem_bytes)
    want = _oracle_program(spec, secs, cols, idx)
    got = _run_placed_and_read(ctx, spec, plan, cols, idx_t)
    for f in range(spec.n_fields):
        assert np.array_equal(got[f], want[f]), f
    small = torch.empty(1024, dtype=torch.uint8, device="cuda")
    with pytest.raises(A.AdhaError):
        A.run_placed(ctx, plan, small, idx_t)
