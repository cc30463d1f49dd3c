"""Programs with branches (CPU only): the oracle's path enumeration pinned by
hand, and the library's expected-cost shortest path against brute force over
every assignment."""
import ctypes
import random

import pytest

from oracle import planner as OP
from paper_1407_4859_amd import adha as A
from paper_1407_4859_amd import synth

IF, ELSE, END = OP.TOK_IF, OP.TOK_ELSE, OP.TOK_END


def test_paths_and_expected_cost_by_hand():
    toks = [0, IF, 1, ELSE, 2, END, 3]
    paths = OP.flow_paths(toks, [0.25])
    assert paths == [(0.25, [("s", 0), ("s", 1), ("j", 0), ("s", 3)]),
                     (0.75, [("s", 0), ("s", 2), ("j", 0), ("s", 3)])]
    # two candidates; remaps cost 10; section costs by hand
    T = [[1, 2], [5, 1], [1, 9], [3, 3]]
    R = [[0, 10], [10, 0]]
    # all in candidate 0: 1 + 0.25*5 + 0.75*1 + 3 = 6
    assert OP.flow_expected_cost(toks, [0.25], T, R, None, 0, [0, 0, 0, 0], [0]) == 6.0
    # section 1 in candidate 1, join back to 0: + 0.25*(10 - 4 + 10) = 10
    assert OP.flow_expected_cost(toks, [0.25], T, R, None, 0, [0, 1, 0, 0], [0]) == 10.0
    best = OP.flow_bruteforce(toks, [0.25], T, R)
    assert best[0] == 6.0
    # nested branches, an empty second part, a start cost
    toks2 = [IF, 0, IF, 1, END, END, 2]
    p2 = OP.flow_paths(toks2, [0.5, 0.2])
    assert sorted(round(p, 12) for p, _ in p2) == [0.1, 0.4, 0.5]
    # all in candidate 1 (start cost 0): 0.5 * (2 + 0.2 * 1 + 9) + 0.5 * 9
    assert OP.flow_expected_cost(toks2, [0.5, 0.2], T, R, [7, 0], 1, [1, 1, 1], [1, 1]) == \
        pytest.approx(0.5 * (2 + 0.2 * 1 + 9) + 0.5 * 9, abs=1e-12)


def _rand_flow(rng, k):
    """A random structured token list over sections 0..k-1 (in order)."""
    toks, probs = [], []
    secs = list(range(k))

    def seq(depth, budget):
        while secs and budget > 0:
            if depth < 2 and rng.random() < 0.35:
                toks.append(IF)
                probs.append(rng.choice([0.0, 0.25, 0.5, 0.75, 1.0]))
                seq(depth + 1, rng.randint(0, 2))
                if rng.random() < 0.7:
                    toks.append(ELSE)
                    seq(depth + 1, rng.randint(0, 2))
                toks.append(END)
            else:
                toks.append(secs.pop(0))
            budget -= 1

    seq(0, 99)
    return toks, probs


def test_flow_solve_matches_bruteforce():
    rng = random.Random(3)
    for _ in range(120):
        k = rng.randint(1, 5)
        C = rng.randint(1, 3)
        toks, probs = _rand_flow(rng, k)
        T = [[float(rng.randint(0, 30)) for _ in range(C)] for _ in range(k)]
        R = [[0.0 if a == b else float(rng.randint(1, 30)) for b in range(C)] for a in range(C)]
        R0 = [float(rng.randint(0, 20)) for _ in range(C)] if rng.random() < 0.5 else None
        if len(probs) > 3 or C ** (1 + k + len(probs)) > 30000:
            continue
        cost, start, node, join = A.flow_solve(T, R, toks, probs, R0)
        best = OP.flow_bruteforce(toks, probs, T, R, R0)
        assert cost == pytest.approx(best[0], abs=1e-9), (toks, probs)
        assert OP.flow_expected_cost(toks, probs, T, R, R0, start, node, join) == pytest.approx(cost, abs=1e-9)


def test_flow_without_branches_is_the_chain():
    rng = random.Random(5)
    for _ in range(50):
        k, C = rng.randint(1, 6), rng.randint(1, 5)
        T = [[float(rng.randint(0, 40)) for _ in range(C)] for _ in range(k)]
        R = [[0.0 if a == b else float(rng.randint(0, 40)) for b in range(C)] for a in range(C)]
        cost, _, node, _ = A.flow_solve(T, R, list(range(k)))
        assert cost == OP.pdl_dp(T, R)[0]


def test_flow_validation_and_analytic_plans():
    spec = synth.config3_struct(1 << 12)
    st = A.Struct.from_spec(spec)
    secs = synth.random_program(3, spec.n_fields, k=6)
    prog = A.Program(st, [A.Section.from_spec(st, s) for s in secs])
    for toks, probs in (([0, 1, 2, 3, 4], []), ([0, 0, 1, 2, 3, 4, 5], []), ([0, IF, 1, 2, 3, 4, 5], [0.5]),
                        ([0, END, 1, 2, 3, 4, 5], []), ([IF, 0, ELSE, 1, ELSE, 2, END, 3, 4, 5], [0.5]),
                        ([IF, 0, END, 1, 2, 3, 4, 5], [1.5]), ([IF, 0, END, 1, 2, 3, 4, 5], [])):
        with pytest.raises(A.AdhaError):
            prog.set_flow(toks, probs)
    toks = [0, IF, 1, 2, ELSE, 3, END, 4, 5]
    prog.set_flow(toks, [0.3])
    opts = A.plan_opts(cost=A.COST_ANALYTIC, cap_bytes=64)
    h = ctypes.c_void_p()
    A.check(A.lib().adha_plan_create(None, prog.h, ctypes.byref(opts), None, 0, None, ctypes.byref(h)))
    pl = A.Plan(h, len(secs))
    T, R = pl.tables()
    cost, start, node, join = A.flow_solve(T, R, toks, [0.3])
    assert pl.choices() == node and pl.joins(1) == join
    assert pl.cost == pytest.approx(cost, rel=1e-12)
    assert OP.flow_expected_cost(toks, [0.3], T, R, None, start, node, join) == pytest.approx(cost, rel=1e-12)
    prog.set_flow([])                                   # back to the plain sequence
    h2 = ctypes.c_void_p()
    A.check(A.lib().adha_plan_create(None, prog.h, ctypes.byref(opts), None, 0, None, ctypes.byref(h2)))
    assert A.Plan(h2, len(secs)).cost == pytest.approx(OP.pdl_dp(T, R)[0], rel=1e-12)
