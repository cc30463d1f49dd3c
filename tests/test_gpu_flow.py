"""Programs with branches on the GPU: the plan is the expected-cost shortest
path over its own measured tables, and every branch outcome runs to the
oracle's result for the sections on that path."""
import itertools

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

IF, ELSE, END = A.TOK_IF, A.TOK_ELSE, A.TOK_END
FLOW = [0, 1, IF, 2, 3, ELSE, 4, END, 5, IF, 6, END, 7]
PROBS = [0.6, 0.3]


@pytest.fixture(scope="module")
def ctx():
    return A.Ctx(0)


def _sections_on_path(taken):
    # the sections the flow runs for these outcomes, in order
    out = [0, 1]
    out += [2, 3] if taken[0] else [4]
    out += [5]
    out += [6] if taken[1] else []
    out += [7]
    return out


@pytest.mark.parametrize("n", [3001, 1 << 16])
def test_flow_plans_run_every_outcome(ctx, n):
    spec = synth.config3_struct(n)
    st = A.Struct.from_spec(spec)
    secs = synth.random_program(3, spec.n_fields)
    prog = A.Program(st, [A.Section.from_spec(st, s) for s in secs])
    prog.set_flow(FLOW, PROBS)
    cols = synth.record_matrix(3, n, spec.dtypes, spec.elem_bytes)
    idx = synth.uniform_index(3, 999, n * 16, n)
    idx_d = torch.from_numpy(idx).cuda()
    plan = A.Plan.create(ctx, prog, A.plan_opts(cost=A.COST_MEASURED, catalogue=A.CAT_FULL, reps=3), idx=idx_d)
    T, R = plan.tables()
    cost, start, node, join = A.flow_solve(T, R, FLOW, PROBS)
    assert plan.choices() == node and plan.joins(2) == join
    assert plan.cost == pytest.approx(cost, rel=1e-12)
    assert OP.flow_expected_cost(FLOW, PROBS, T, R, None, start, node, join) == pytest.approx(cost, rel=1e-9)
    say("flow plan", n, "choices", node, "joins", join, "expected us", round(cost, 1))
    plans = [("planned", plan), ("aos", A.Plan.uniform(prog, A.Layout.aos(st))),
             ("soa", A.Plan.uniform(prog, A.Layout.soa(st)))]
    cap = max(plan.candidate(c).nbytes for c in range(plan.n_candidates)) + 256
    for taken in itertools.product([0, 1], repeat=2):
        Oa = oaos(n, spec.elem_bytes)
        want = oracle.pack(Oa, cols)
        for s in _sections_on_path(taken):
            x = secs[s]
            oracle.section(Oa, spec.dtypes, x.op, x.read, x.write, x.degree, idx if x.degree else None, want)
        for name, pl in plans:
            first = pl.candidate(pl.choices()[0])
            gof, tiles = first.groups(spec.n_fields)
            O1 = OLayout(n, spec.elem_bytes, gof, tiles)
            a = dev_bytes(oracle.pack(O1, cols), extra=cap - O1.nbytes)
            b = torch.empty(cap, dtype=torch.uint8, device="cuda")
            say("flow run", n, name, "taken", taken)
            out_h, in_b = A.run_flow(ctx, pl, first, a, b, taken, idx_d)
            ctx.check()
            cands = [pl.candidate(c) for c in range(pl.n_candidates)]
            L = [c for c in cands + [first] if c.h.value == out_h][0]
            gof, tiles = L.groups(spec.n_fields)
            O = OLayout(n, spec.elem_bytes, gof, tiles)
            got = oracle.remap(O, host(b if in_b else a, O.nbytes), Oa)
            assert np.array_equal(got, want), (name, taken)
    with pytest.raises(A.AdhaError):
        first = plan.candidate(plan.choices()[0])
        A.run(ctx, plan, first, torch.empty(cap, dtype=torch.uint8, device="cuda"),
              torch.empty(cap, dtype=torch.uint8, device="cuda"), idx_d)
