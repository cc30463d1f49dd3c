"""GPU parity of reduction sections against the oracle.

The oracle's floating-point cells are the exact sums rounded once
(math.fsum).  The device adds with compensation (double-double) in a fixed
order, so every F32 and F64 cell must lie within 1 ulp of the oracle's --
on the generator's plain values, on values spread over 81 binades (2^-40 to
2^41) and under heavy cancellation -- and two runs must give the same bits.
I32 cells and the counts must match exactly."""
import numpy as np
import pytest
import torch

import oracle
from oracle import reduce as OR
from oracle.layout import Layout as OLayout, aos as oaos, soa as osoa, from_partition
from paper_1407_4859_amd import adha as A
from paper_1407_4859_amd import synth
from gpu_util import dev_bytes, host, mirror, say

pytestmark = pytest.mark.gpu

F32, F64, I32 = synth.F32, synth.F64, synth.I32


@pytest.fixture(scope="module")
def ctx():
    return A.Ctx(0)


def _struct(n, seed, n_keys, bad=()):
    """Fields: 0-5 f32, 6 key (i32 in [0, n_keys)), 7 i32, 8-9 f64, 10 f32."""
    dtypes = [F32] * 6 + [I32, I32, F64, F64, F32]
    eb = [4] * 8 + [8, 8, 4]
    cols = synth.record_matrix(seed, n, dtypes, eb)
    keys = synth.uniform_index(seed, 77, n, n_keys).astype(np.int32)
    for r, k in bad:
        keys[r] = k
    cols[6] = keys.view(np.uint8).reshape(n, 4)
    return synth.StructSpec(n, dtypes, eb), cols


def ulps64(a: float, b: float) -> int:
    """Distance in units in the last place between two doubles."""
    def ordered(x):
        i = int(np.array([x], np.float64).view(np.int64)[0])
        return i if i >= 0 else -(i & 0x7FFFFFFFFFFFFFFF)
    return abs(ordered(a) - ordered(b))


def _check(got_cells, table, dtypes, read, values=None):
    """got_cells: uint64 cells from the device; table: the oracle's.
    Floating-point cells within 1 ulp of the oracle's, the rest exact.
    Returns the largest ulp distance seen."""
    want = OR.table_cells(table, dtypes, read)
    cols = len(read) + 1
    worst = 0
    for k, row in enumerate(table):
        for j in range(cols):
            g, w = got_cells[k * cols + j], want[k * cols + j]
            if j < len(read) and dtypes[read[j]] != I32:
                gv = float(np.array([g], np.uint64).view(np.float64)[0])
                u = ulps64(gv, row[j])
                worst = max(worst, u)
                assert u <= 1, (k, j, gv, row[j], u)
            else:
                assert g == w, (k, j, int(g), int(w))
    return worst


def _run(ctx, spec, cols, O, read, key, n_keys):
    st = A.Struct.from_spec(spec)
    L = mirror(st, O)
    buf_h = oracle.pack(O, cols)
    dev = dev_bytes(buf_h)
    cells = n_keys * (len(read) + 1)
    out = torch.full((cells * 8,), 0xEE, dtype=torch.uint8, device="cuda")
    sec = A.Section.reduce(st, read, key, n_keys, out)
    A.section_run(ctx, sec, L, dev)
    return buf_h, sec, out


@pytest.mark.parametrize("n", [1, 255, 4096 + 13, 1 << 18])
def test_reduce_matches_oracle_on_layouts(ctx, n):
    spec, cols = _struct(n, 5, 5)
    eb = spec.elem_bytes
    read = [0, 2, 5, 7, 8, 10]
    layouts = (oaos(n, eb), osoa(n, eb), OLayout(n, eb, [0] * 11, [64]),
               from_partition(n, eb, [[0, 2, 5, 6], [7, 8, 9, 10]], 1),
               from_partition(n, eb, [[0, 6], [2, 5, 8]], 16))
    for O in layouts:
        say("reduce", n, O)
        buf_h, sec, out = _run(ctx, spec, cols, O, read, 6, 5)
        ctx.check()
        table, bad = OR.reduce(O, spec.dtypes, read, 6, 5, buf_h)
        assert bad == 0
        got = host(out).view(np.uint64)
        _check(got, table, spec.dtypes, read)


@pytest.mark.parametrize("n_keys", [1, 2, 5, 8])
def test_reduce_f32_reads_on_every_layout_kind(ctx, n_keys):
    """All-F32 read sets (the straight-line register kernel) on interleaved,
    single-field, tiled and grouped-tiled layouts, ragged N, with and
    without a key field."""
    n = 3 * 4096 + 77
    spec, cols = _struct(n, 9, n_keys)
    eb = spec.elem_bytes
    read = [0, 1, 2, 3, 4, 5, 10]
    key = -1 if n_keys == 1 else 6
    for O in (oaos(n, eb), osoa(n, eb), OLayout(n, eb, [0] * 11, [64]),
              from_partition(n, eb, [[0, 1, 6], [2, 3, 4, 5, 10]], 4),
              from_partition(n, eb, [[0, 6], [2, 5, 8]], 16)):
        say("reduce f32", n_keys, O)
        buf_h, sec, out = _run(ctx, spec, cols, O, read, key, n_keys)
        ctx.check()
        table, bad = OR.reduce(O, spec.dtypes, read, key, n_keys, buf_h)
        assert bad == 0
        _check(host(out).view(np.uint64), table, spec.dtypes, read, {})


@pytest.mark.parametrize("n_keys,read", [(1, [0, 1, 7, 9]), (1, [0, 1, 2]), (2, [0, 7, 8, 10]), (3, [1, 2, 3, 4, 5]),
                                         (6, [0, 2, 7, 9, 10]), (7, [0, 1, 2, 3, 4, 5, 7, 10]),
                                         (8, [0, 1, 7, 8, 9, 10]), (9, [0, 1, 7]), (64, [0, 1, 2, 3]),
                                         (128, list(range(6)) + [7] + [8, 9, 10]),
                                         (409, [0, 1, 2, 3, 4, 5, 7, 8, 10])])
def test_reduce_key_counts_and_no_key(ctx, n_keys, read):
    n = 100_000
    spec, cols = _struct(n, 6, n_keys)
    O = osoa(n, spec.elem_bytes)
    key = -1 if n_keys == 1 else 6
    say("reduce keys", n_keys, "read", read)
    buf_h, sec, out = _run(ctx, spec, cols, O, read, key, n_keys)
    ctx.check()
    table, _ = OR.reduce(O, spec.dtypes, read, key, n_keys, buf_h)
    _check(host(out).view(np.uint64), table, spec.dtypes, read)


def test_reduce_bad_keys_are_left_out_and_reported(ctx):
    n = 10_000
    spec, cols = _struct(n, 7, 8, bad=[(0, -1), (17, 8), (9999, 1 << 30)])
    O = oaos(n, spec.elem_bytes)
    buf_h, sec, out = _run(ctx, spec, cols, O, [0, 7], 6, 8)
    with pytest.raises(A.AdhaError) as e:
        ctx.check()
    assert e.value.status == A.ERR_INVALID
    ctx.check()                                      # the flag is cleared
    table, bad = OR.reduce(O, spec.dtypes, [0, 7], 6, 8, buf_h)
    assert bad == 3 and sum(r[-1] for r in table) == n - 3
    _check(host(out).view(np.uint64), table, spec.dtypes, [0, 7], {})


def test_reduce_overlap_is_rejected_and_empty_struct_zeroes(ctx):
    spec, cols = _struct(1000, 8, 4)
    st = A.Struct.from_spec(spec)
    O = oaos(1000, spec.elem_bytes)
    L = mirror(st, O)
    dev = dev_bytes(oracle.pack(O, cols), extra=4096)
    sec = A.Section.reduce(st, [0, 1], 6, 4, dev[O.nbytes - 256:])   # table inside the data
    with pytest.raises(A.AdhaError):
        A.section_run(ctx, sec, L, dev)
    st0 = A.Struct(0, spec.dtypes, spec.elem_bytes)
    out = torch.full((4 * 3 * 8,), 0xEE, dtype=torch.uint8, device="cuda")
    s0 = A.Section.reduce(st0, [0, 1], 6, 4, out)
    A.section_run(ctx, s0, A.Layout.aos(st0), torch.empty(256, dtype=torch.uint8, device="cuda"))
    ctx.check()
    assert not host(out).any()


def test_program_with_a_reduction_runs_to_the_oracle_result(ctx):
    # a K-Means-like pair: a direct section writes field 10, then the
    # reduction reads it together with other fields, per key
    n = (1 << 16) + 3
    spec, cols = _struct(n, 9, 5)
    st = A.Struct.from_spec(spec)
    cells = 5 * 6
    out = torch.zeros(cells * 8, dtype=torch.uint8, device="cuda")
    g = A.Section(st, A.OP_GEN, [0, 1, 2, 3], [10], 0)
    r = A.Section.reduce(st, [0, 4, 7, 9, 10], 6, 5, out)
    prog = A.Program(st, [g, r])
    plan = A.Plan.create(ctx, prog, A.plan_opts(cost=A.COST_MEASURED, catalogue=A.CAT_FULL, reps=3))
    say("program with reduction: plan", plan.choices(), "of", plan.n_candidates)
    assert not host(out).any()                       # planning left the table alone
    Oa = oaos(n, spec.elem_bytes)
    want_buf = oracle.pack(Oa, cols)
    oracle.section(Oa, spec.dtypes, A.OP_GEN, [0, 1, 2, 3], [10], 0, None, want_buf)
    table, _ = OR.reduce(Oa, spec.dtypes, [0, 4, 7, 9, 10], 6, 5, want_buf)
    for pl in (plan, A.Plan.uniform(prog, A.Layout.aos(st)), A.Plan.uniform(prog, A.Layout.soa(st))):
        first = pl.candidate(pl.choices()[0])
        gof, tiles = first.groups(spec.n_fields)
        O1 = OLayout(n, spec.elem_bytes, gof, tiles)
        cap = max(pl.candidate(c).nbytes for c in range(pl.n_candidates)) + 256
        a = dev_bytes(oracle.pack(O1, cols), extra=cap - O1.nbytes)
        b = torch.empty(cap, dtype=torch.uint8, device="cuda")
        out.zero_()
        A.run(ctx, pl, first, a, b)
        ctx.check()
        _check(host(out).view(np.uint64), table, spec.dtypes, [0, 4, 7, 9, 10])


@pytest.mark.timeout(900)
def test_kmeans_workload_full_size(ctx):
    """The K-Means-shaped program at its full size (2^23 points): the planned,
    all-AoS and all-SoA runs give the oracle's table."""
    import os
    from concurrent.futures import ThreadPoolExecutor
    from gpu_util import fill_aos_device
    n = 8388608
    spec = synth.kmeans_struct(n)
    st = A.Struct.from_spec(spec)
    gen_spec, (rd, key, nk) = synth.kmeans_sections()
    say("kmeans full: generating", n, "points on the device")
    src = fill_aos_device(spec, 6)
    S = spec.record_bytes
    src[: n * S].view(n, S)[:, 4 * key:4 * key + 4] = \
        synth.uniform_index_torch(6, 77, n, nk, "cuda").view(torch.uint8).view(n, 4)
    want = src.cpu().numpy()
    O = oaos(n, spec.elem_bytes)
    assert O.nbytes == want.size
    cores = max(1, min(16, len(os.sched_getaffinity(0))))
    bounds = [n * i // cores for i in range(cores + 1)]
    say("kmeans full: oracle loop on", cores, "threads")
    with ThreadPoolExecutor(cores) as ex:
        list(ex.map(lambda i: oracle.section(O, spec.dtypes, gen_spec.op, gen_spec.read, gen_spec.write, 0, None,
                                             want, bounds[i], bounds[i + 1]), range(cores)))
    say("kmeans full: oracle reduction")
    table, bad = OR.reduce(O, spec.dtypes, rd, key, nk, want)
    assert bad == 0 and sum(r[-1] for r in table) == n
    out = torch.zeros(nk * (len(rd) + 1) * 8, dtype=torch.uint8, device="cuda")
    prog = A.Program(st, [A.Section.from_spec(st, gen_spec), A.Section.reduce(st, rd, key, nk, out)])
    La = A.Layout.aos(st)
    cap = max(La.nbytes, A.Layout.soa(st).nbytes) + (1 << 26)
    buf_a = torch.empty(cap, dtype=torch.uint8, device="cuda")
    buf_b = torch.empty(cap, dtype=torch.uint8, device="cuda")
    plans = [("planned", A.Plan.create(ctx, prog, A.plan_opts(cost=A.COST_MEASURED, catalogue=A.CAT_FULL,
                                                             reps=3))),
             ("all-AoS", A.Plan.uniform(prog, La)), ("all-SoA", A.Plan.uniform(prog, A.Layout.soa(st)))]
    for name, plan in plans:
        say("kmeans full: run", name, plan.choices())
        buf_a[: La.nbytes].copy_(src)
        out.zero_()
        A.run(ctx, plan, La, buf_a, buf_b)
        ctx.check()
        _check(host(out).view(np.uint64), table, spec.dtypes, rd, {})


def _wide_struct(n, seed, n_keys, cancel):
    """Fields: 0-2 f32, 3 key, 4-5 f64, 6 i32.  F32 and F64 values are
    +-(1 + m) * 2^E with E in [-40, 40] (81 binades).  cancel: the records
    come in pairs with one key, the second of a pair the negation of the
    first, except that both records of every 8th pair hold values with E
    in [4, 14]; the sum of a key is then the sum of those few small values
    while sum|x| is some 2^30 - 2^34 times larger."""
    dtypes = [F32, F32, F32, I32, F64, F64, I32]
    eb = [4, 4, 4, 4, 8, 8, 4]
    cols = []
    for f, (dt, e) in enumerate(zip(dtypes, eb)):
        z = synth.splitmix64(seed, f, 0, n)
        if dt == I32:
            cols.append(synth.decode(z, dt, e))
            continue
        wide = synth.decode_wide(z, dt).view(np.float32 if dt == F32 else np.float64).reshape(-1).copy()
        if cancel:
            small = synth.decode_wide(z, dt, 4, 14).view(wide.dtype).reshape(-1)
            pair = np.arange(n) // 2
            odd = (np.arange(n) % 2 == 1) & (np.arange(n) < n - n % 2)
            resid = pair % 8 == 7
            wide[odd & ~resid] = -wide[np.nonzero(odd & ~resid)[0] - 1]
            wide[resid] = small[resid]
        cols.append(np.ascontiguousarray(wide).view(np.uint8).reshape(n, e))
    keys = synth.uniform_index(seed, 77, n, n_keys).astype(np.int32)
    if cancel:
        keys[1::2] = keys[0:n - n % 2:2][: len(keys[1::2])]
    cols[3] = keys.view(np.uint8).reshape(n, 4)
    return synth.StructSpec(n, dtypes, eb), cols


@pytest.mark.parametrize("n_keys", [1, 2, 3, 4, 5, 6, 7, 8, 9, 64, 409])
@pytest.mark.parametrize("cancel", [False, True])
def test_reduce_wide_values_within_one_ulp_and_repeatable(ctx, n_keys, cancel):
    """General F32 / F64 values over 81 binades, with and without heavy
    cancellation, every key-count form: each cell within 1 ulp of the exactly
    rounded sum; a second run gives the same bytes."""
    n = (1 << 16) + 37
    spec, cols = _wide_struct(n, 40 + n_keys % 200, n_keys, cancel)
    key = -1 if n_keys == 1 else 3
    worst = 0
    for read in ([0, 1, 2, 4, 5, 6], [0, 1, 2]):
        for O in (osoa(n, spec.elem_bytes), oaos(n, spec.elem_bytes)):
            say("reduce wide", n_keys, "cancel", cancel, "read", read, O)
            buf_h, sec, out = _run(ctx, spec, cols, O, read, key, n_keys)
            ctx.check()
            first = host(out).copy()
            table, bad = OR.reduce(O, spec.dtypes, read, key, n_keys, buf_h)
            assert bad == 0
            worst = max(worst, _check(first.view(np.uint64), table, spec.dtypes, read))
            out.fill_(0x33)
            A.section_run(ctx, sec, mirror(A.Struct.from_spec(spec), O), dev_bytes(buf_h))
            ctx.check()
            assert np.array_equal(host(out), first), "second run differs"
    say("reduce wide", n_keys, "cancel", cancel, "largest ulp distance", worst)


def test_reduce_plain_option_is_repeatable_and_bounded(ctx):
    """ADHA_OPT_REDUCE_COMPENSATED = 0: plain double sums in the same fixed
    order -- repeatable, within (m-1) 2^-53 sum|x| of the exact sum."""
    n = (1 << 16) + 37
    c2 = A.Ctx(0)
    c2.set_option(A.OPT_REDUCE_COMPENSATED, 0)
    for n_keys, read in ((5, [0, 1, 2, 4, 5, 6]), (64, [0, 1, 2, 4, 5, 6]), (5, [0, 1, 2])):
        spec, cols = _wide_struct(n, 7, n_keys, False)
        O = osoa(n, spec.elem_bytes)
        buf_h, sec, out = _run(c2, spec, cols, O, read, 3, n_keys)
        c2.check()
        first = host(out).copy()
        A.section_run(c2, sec, mirror(A.Struct.from_spec(spec), O), dev_bytes(buf_h))
        c2.check()
        assert np.array_equal(host(out), first)
        table, _ = OR.reduce(O, spec.dtypes, read, 3, n_keys, buf_h)
        keys = OR.field_values(O, buf_h, I32, 3)
        got = first.view(np.float64)
        for k in range(n_keys):
            for j, f in enumerate(read):
                if spec.dtypes[f] == I32:
                    continue
                v = np.abs(OR.field_values(O, buf_h, spec.dtypes[f], f)[keys == k].astype(np.float64))
                bound = max(len(v) - 1, 0) * 2.0 ** -53 * float(v.sum()) * (1 + 1e-12)
                assert abs(got[k * (len(read) + 1) + j] - table[k][j]) <= bound
