"""Plans over the GPU and the host (section 2: each section is mapped to a
device).  Explicit plans exercise every kind of move between the devices
and layouts; measured plans are checked against the shortest path over their
own node tables; every run ends with the oracle's data."""
import numpy as np
import pytest
import torch

import oracle
from oracle import planner as OP
from oracle import reduce as OR
from oracle.layout import Layout as OLayout, aos as oaos, soa as osoa
from paper_1407_4859_amd import adha as A
from paper_1407_4859_amd import synth
from gpu_util import host, mirror, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    c = A.Ctx(0)
    c.set_option(A.OPT_HOST_THREADS, 8)
    return c


def _olayout(spec, lay):
    gof, tiles = lay.groups(spec.n_fields)
    return OLayout(spec.n, spec.elem_bytes, gof, tiles)


def _oracle_program(spec, secs, cols, idx):
    O = oaos(spec.n, spec.elem_bytes)
    buf = oracle.pack(O, cols)
    for s in secs:
        oracle.section(O, spec.dtypes, s.op, s.read, s.write, s.degree, idx if s.degree else None, buf)
    return O, buf


def _buffers(cap):
    dev = [torch.empty(cap, dtype=torch.uint8, device="cuda") for _ in range(2)]
    hst = [torch.empty(cap, dtype=torch.uint8).pin_memory() for _ in range(2)]
    return dev, hst


def _final_aos(ctx, spec, plan, out_h, out_dev, in_b, dev, hst, st):
    """The data at the end of a run, as the packed record image (host)."""
    cands = [plan.candidate(c) for c in range(plan.n_candidates)]
    L = [c for c in cands if c.h.value == out_h][0]
    O = _olayout(spec, L)
    raw = (hst if out_dev == 1 else dev)[1 if in_b else 0]
    buf = raw.cpu().numpy()[: O.nbytes] if out_dev == 0 else raw.numpy()[: O.nbytes].copy()
    return oracle.remap(O, buf, oaos(spec.n, spec.elem_bytes))


@pytest.mark.parametrize("n", [1000, (1 << 15) + 3])
def test_explicit_plans_cover_every_move(ctx, n):
    spec = synth.config3_struct(n)
    st = A.Struct.from_spec(spec)
    secs = synth.random_program(3, spec.n_fields)
    prog = A.Program(st, [A.Section.from_spec(st, s) for s in secs])
    cols = synth.record_matrix(3, n, spec.dtypes, spec.elem_bytes)
    idx = synth.uniform_index(3, 999, n * 16, n)
    Ow, want = _oracle_program(spec, secs, cols, idx)
    osecs = [(s.read, s.write, s.degree) for s in secs]
    cat = OP.catalogue(osecs, n, spec.elem_bytes, 64)
    pick = [cat[i % len(cat)] for i in (0, 1, 2, 5, 9, 14, 20, 33)]
    L = [mirror(st, O) for O in pick]
    # devices: stay, GPU->host with and without a layout change, host->host,
    # host->GPU with a layout change, GPU->GPU
    plans = [[0, 1, 1, 0, 0, 1, 0, 1], [1, 1, 0, 1, 0, 0, 1, 1], [1] * 8]
    layouts_same = [L[0], L[0], L[3], L[3], L[3], L[6], L[6], L[1]]
    cap = max(O.nbytes for O in cat) + 256
    dev, hst = _buffers(cap)
    idx_d = torch.from_numpy(idx).cuda()
    for devices in plans:
        for lays in (L, layouts_same):
            plan = A.Plan.explicit(prog, lays, devices)
            assert plan.devices() == devices
            for in_device in (0, 1):
                O0 = _olayout(spec, lays[0])
                img = oracle.pack(O0, cols)
                if in_device == 0:
                    dev[0][: O0.nbytes].copy_(torch.from_numpy(img))
                else:
                    hst[0][: O0.nbytes].copy_(torch.from_numpy(img))
                say("hetero explicit", n, devices, "start", in_device)
                out_h, out_d, in_b = A.run_hetero(ctx, plan, lays[0], in_device, dev[0], dev[1], hst[0], hst[1],
                                                  idx_d, idx)
                ctx.check()
                torch.cuda.synchronize()
                assert out_d == devices[-1]
                got = _final_aos(ctx, spec, plan, out_h, out_d, in_b, dev, hst, None)
                assert np.array_equal(got, want), (devices, in_device)
    with pytest.raises(A.AdhaError):             # GPU-only runs refuse host sections
        A.run(ctx, A.Plan.explicit(prog, L, plans[0]), L[0], dev[0], dev[1], idx_d)


def test_measured_plans_over_both_devices(ctx):
    for spec, secs, seed in ((synth.config1_struct(65536), synth.config1_sections(), 1),
                             (synth.config3_struct(1 << 14), synth.random_program(7, 32), 7),
                             (synth.config3_struct(512), synth.random_program(8, 32), 8)):
        n = spec.n
        st = A.Struct.from_spec(spec)
        prog = A.Program(st, [A.Section.from_spec(st, s) for s in secs])
        cols = synth.record_matrix(seed, n, spec.dtypes, spec.elem_bytes)
        idx = synth.uniform_index(seed, 999, n * 16, n)
        idx_d = torch.from_numpy(idx).cuda()
        Ow, want = _oracle_program(spec, secs, cols, idx)
        for init in (A.INIT_FREE, A.INIT_HOST_AOS):
            plan = A.Plan.create(ctx, prog, A.plan_opts(cost=A.COST_MEASURED, catalogue=A.CAT_FULL, reps=3,
                                                        devices=A.DEVICES_GPU_HOST, init=init), idx=idx_d)
            T, R = plan.node_tables()
            C = plan.n_candidates
            R0 = [0.0 if m == C else R[C][m] for m in range(2 * C)] if init == A.INIT_HOST_AOS else None
            cost, path = OP.pdl_dp(T, R, R0)
            assert [m % C for m in path] == plan.choices() and [int(m >= C) for m in path] == plan.devices()
            assert plan.cost == pytest.approx(cost, rel=1e-12)
            say("hetero measured n", n, "init", init, "devices", plan.devices(), "choices", plan.choices(),
                "cost us", round(plan.cost, 1))
            cap = max(plan.candidate(c).nbytes for c in range(C)) + 256
            dev, hst = _buffers(cap)
            start = A.Layout.aos(st)
            in_device = 1 if init == A.INIT_HOST_AOS else plan.devices()[0]
            img = oracle.pack(oaos(n, spec.elem_bytes), cols)
            (hst if in_device == 1 else dev)[0][: img.size].copy_(torch.from_numpy(img))
            out_h, out_d, in_b = A.run_hetero(ctx, plan, start, in_device, dev[0], dev[1], hst[0], hst[1],
                                              idx_d, idx)
            ctx.check()
            torch.cuda.synchronize()
            cands = [plan.candidate(c) for c in range(C)]
            Lend = [c for c in cands + [start] if c.h.value == out_h][0]
            O = _olayout(spec, Lend)
            raw = (hst if out_d == 1 else dev)[1 if in_b else 0]
            buf = raw.cpu().numpy()[: O.nbytes].copy()
            assert np.array_equal(oracle.remap(O, buf, oaos(n, spec.elem_bytes)), want)


def test_host_reduction_and_bad_indices(ctx):
    n = 20000
    dtypes = [synth.F32] * 4 + [synth.I32, synth.I32, synth.F32]
    eb = [4] * 7
    cols = synth.record_matrix(9, n, dtypes, eb)
    keys = synth.uniform_index(9, 77, n, 5).astype(np.int32)
    cols[4] = keys.view(np.uint8).reshape(n, 4)
    spec = synth.StructSpec(n, dtypes, eb)
    st = A.Struct.from_spec(spec)
    out = torch.zeros(5 * 5 * 8, dtype=torch.uint8, device="cuda")
    g = A.Section(st, A.OP_GEN, [0, 1, 2], [6], 0)
    r = A.Section.reduce(st, [0, 3, 5, 6], 4, 5, out)
    prog = A.Program(st, [g, r])
    soa = A.Layout.soa(st)
    plan = A.Plan.explicit(prog, [soa, A.Layout.aos(st)], [0, 1])
    Oa = oaos(n, eb)
    want = oracle.pack(Oa, cols)
    oracle.section(Oa, dtypes, synth.OP_GEN, [0, 1, 2], [6], 0, None, want)
    table, _ = OR.reduce(Oa, dtypes, [0, 3, 5, 6], 4, 5, want)
    dev, hst = _buffers(Oa.nbytes + 4096)
    img = oracle.pack(osoa(n, eb), cols)
    dev[0][: img.size].copy_(torch.from_numpy(img))
    A.run_hetero(ctx, plan, soa, 0, dev[0], dev[1], hst[0], hst[1])
    ctx.check()
    got = host(out).view(np.uint64)
    assert np.array_equal(got, OR.table_cells(table, dtypes, [0, 3, 5, 6]))
    # a host gather meeting out-of-range indices reports them
    gs = A.Section(st, A.OP_GEN, [0, 1], [2], 4)
    p2 = A.Plan.explicit(A.Program(st, [gs]), [soa], [1])
    idx = synth.uniform_index(9, 5, n * 4, n)
    idx[11] = -1
    hst[0][: img.size].copy_(torch.from_numpy(img))
    A.run_hetero(ctx, p2, soa, 1, dev[0], dev[1], hst[0], hst[1], None, idx)
    with pytest.raises(A.AdhaError):
        ctx.check()
    ctx.check()
