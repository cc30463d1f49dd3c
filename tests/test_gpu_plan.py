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
