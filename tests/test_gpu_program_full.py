"""Full-size parity of the multi-section program workload.

The workload is 2^24 records of 144 bytes (20 f32, 8 i32, 4 f64) with 8 GEN
sections. Four of them gather 16 uniform neighbours from a 1 GiB index array.
The planned run on the device is compared with the oracle over the whole
struct. The oracle runs on the host cores over record ranges; records are
independent within a section, and a gather never writes a field it reads.

The plans are the one the benchmark builds and times (the full catalogue
with measured costs, so remaps happen between runs) and the analytic-cost
plan; the all-SoA and all-AoS uniform plans are checked too.
Every plan runs placed in one arena (adha_run_placed), the executor the
benchmark times: between sections only the groups that change are moved.
Device results are remapped back to the packed record image on the device
and compared byte for byte; a floating-point field may differ by at most
1 ulp."""
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest
import torch

import oracle
from oracle.layout import aos as oaos
from paper_1407_4859_amd import adha as A
from paper_1407_4859_amd import synth
from gpu_util import fill_aos_device, say
from test_gpu_section import ulp_distance

pytestmark = pytest.mark.gpu

N = 1 << 24


@pytest.fixture(scope="module")
def ctx():
    return A.Ctx(0)


def _cores():
    try:
        return max(1, min(16, len(os.sched_getaffinity(0))))
    except AttributeError:
        return 1


def test_device_fill_is_the_packed_record_image():
    spec = synth.config3_struct(1000)
    dev = fill_aos_device(spec, 3)
    want = synth.pack_aos(synth.record_matrix(3, 1000, spec.dtypes, spec.elem_bytes), 1000).reshape(-1)
    assert np.array_equal(dev.cpu().numpy(), want)
    # the oracle's AoS image is the same bytes followed by zero padding to 256
    O = oaos(1000, spec.elem_bytes)
    img = oracle.pack(O, synth.record_matrix(3, 1000, spec.dtypes, spec.elem_bytes))
    assert O.nbytes == 144128 and np.array_equal(img[: want.size], want) and not img[want.size:].any()


@pytest.mark.timeout(900)
def test_config3_full_size_plans_match_oracle(ctx):
    spec = synth.config3_struct(N)
    eb = spec.elem_bytes
    st = A.Struct.from_spec(spec)
    secs = synth.random_program(3, spec.n_fields)
    prog = A.Program(st, [A.Section.from_spec(st, s) for s in secs])
    say("program full: generating", N, "records on the device")
    src = fill_aos_device(spec, 3)
    idx = synth.uniform_index_torch(3, 999, N * 16, N, "cuda")
    # the oracle's inputs: the same seeded draws, copied to the host
    want = src.cpu().numpy()
    idx_h = idx.cpu().numpy()
    O = oaos(N, eb)
    assert O.nbytes == want.size
    cores = _cores()
    bounds = [N * i // cores for i in range(cores + 1)]
    for s in secs:
        say("program full: oracle", s, "on", cores, "threads")
        with ThreadPoolExecutor(cores) as ex:
            bad = sum(ex.map(lambda i: oracle.section(O, spec.dtypes, s.op, s.read, s.write, s.degree,
                                                      idx_h if s.degree else None, want,
                                                      bounds[i], bounds[i + 1]), range(cores)))
        assert bad == 0
    del idx_h
    La = A.Layout.aos(st)
    back = torch.empty(La.nbytes, dtype=torch.uint8, device="cuda")
    say("program full: planning with measured costs (the benchmark's plan)")
    plans = [("measured", A.Plan.create(ctx, prog, A.plan_opts(cost=A.COST_MEASURED, catalogue=A.CAT_FULL,
                                                              cap_bytes=64), idx=idx)),
             ("analytic", A.Plan.create(ctx, prog, A.plan_opts(cost=A.COST_ANALYTIC, catalogue=A.CAT_FULL,
                                                              cap_bytes=64))),
             ("all-SoA", A.Plan.uniform(prog, A.Layout.soa(st))),
             ("all-AoS", A.Plan.uniform(prog, La))]
    arena = torch.empty(max(A.plan_arena(p)[0] for _, p in plans), dtype=torch.uint8, device="cuda")
    for name, plan in plans:
        arena_bytes, start, end = A.plan_arena(plan)
        say("program full: run", name, plan.choices(), "placed in", arena_bytes, "bytes")
        # the data starts in the plan's start layout at the arena's start
        A.remap(ctx, La, src, start, arena)
        A.run_placed(ctx, plan, arena, idx)
        ctx.check()
        # read the result through the end layout, back into the record image
        A.remap(ctx, end, arena, La, back)
        ctx.check()
        got = back.cpu().numpy()
        if np.array_equal(got, want):
            continue
        g2, w2 = got.reshape(N, -1), want.reshape(N, -1)
        off = 0
        for f, e in enumerate(eb):
            g, w = g2[:, off:off + e], w2[:, off:off + e]
            if not np.array_equal(g, w):
                rows = np.nonzero((g != w).any(axis=1))[0]
                u = ulp_distance(np.ascontiguousarray(g[rows]), np.ascontiguousarray(w[rows]), spec.dtypes[f])
                say("program full:", name, "field", f, "differs at", rows.size, "records, max ulp", u)
                assert u <= 1, (name, f)
            off += e
