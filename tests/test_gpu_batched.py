"""GPU tests of the batched remap (one persistent launch over many arrays,
optionally replayed from a captured graph) and of the autotuner."""
import os
import tempfile

import numpy as np
import pytest
import torch

import oracle
from oracle.layout import Layout as OLayout, aos as oaos
from paper_1407_4859_amd import adha as A
from paper_1407_4859_amd import synth
from gpu_util import dev_bytes, first_diff, host, mirror, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    return A.Ctx(0)


def _arrays(n_arrays, hi_log2, seed=4):
    out = []
    for i, a in enumerate(synth.config4_arrays(seed, n_arrays, 10, hi_log2)):
        eb = a["elem_bytes"]
        st = A.Struct(a["n"], [A.RAW] * len(eb), eb)
        Oa = oaos(a["n"], eb)
        Ob = OLayout(a["n"], eb, a["target_gof"], a["target_tiles"])
        cols = [synth.field_values(seed, 64 * i + f, a["n"], synth.RAW, e) for f, e in enumerate(eb)]
        src_h = oracle.pack(Oa, cols)
        out.append(dict(st=st, Oa=Oa, Ob=Ob, src=dev_bytes(src_h), want=oracle.remap(Oa, src_h, Ob),
                        la=mirror(st, Oa), lb=mirror(st, Ob),
                        dst=torch.full((Ob.nbytes,), 0xA5, dtype=torch.uint8, device="cuda")))
    return out


def _check(arrs, label):
    for i, a in enumerate(arrs):
        d = first_diff(host(a["dst"], a["Ob"].nbytes), a["want"])
        assert d is None, (label, i, d)


def test_batched_matches_oracle_and_graph_replays(ctx):
    arrs = _arrays(48, 15)
    items = [(a["la"], a["src"], a["lb"], a["dst"]) for a in arrs]
    say("batched eager")
    A.remap_batched(ctx, items, 0)
    ctx.check()
    _check(arrs, "eager")
    for rep in range(3):
        for a in arrs:                      # eager work between replays
            a["dst"].fill_(0x5A)
        torch.cuda.synchronize()
        say("batched graph replay", rep)
        A.remap_batched(ctx, items, A.BATCH_GRAPH)
        ctx.check()
        _check(arrs, f"graph {rep}")
    for a in arrs:
        a["dst"].fill_(0)
    A.remap_batched(ctx, items, A.BATCH_SEPARATE)
    ctx.check()
    _check(arrs, "separate")


def test_batched_with_empty_and_tiny_arrays(ctx):
    arrs = []
    for i, (n, eb) in enumerate(((0, [4, 4]), (1, [8, 4, 4]), (63, [4] * 5), (64, [8] * 3), (300, [4, 8]))):
        st = A.Struct(n, [A.RAW] * len(eb), eb)
        Oa = oaos(n, eb)
        Ob = OLayout(n, eb, list(range(len(eb))), [1] * len(eb)) if i % 2 else \
            OLayout(n, eb, [0] * len(eb), [64])
        cols = [synth.field_values(9, 64 * i + f, n, synth.RAW, e) for f, e in enumerate(eb)]
        src_h = oracle.pack(Oa, cols)
        arrs.append(dict(Ob=Ob, src=dev_bytes(src_h), want=oracle.remap(Oa, src_h, Ob),
                         la=mirror(st, Oa), lb=mirror(st, Ob), st=st,
                         dst=torch.full((max(1, Ob.nbytes),), 0xA5, dtype=torch.uint8, device="cuda")))
    items = [(a["la"], a["src"], a["lb"], a["dst"]) for a in arrs]
    A.remap_batched(ctx, items, A.BATCH_GRAPH)
    ctx.check()
    _check(arrs, "tiny")


def test_batched_rejects_overlapping_items(ctx):
    st = A.Struct(1000, [A.F32, A.F32])
    la, ls = A.Layout.aos(st), A.Layout.soa(st)
    buf = torch.zeros(1 << 16, dtype=torch.uint8, device="cuda")
    items = [(la, buf[:8192], ls, buf[16384:24576]), (la, buf[32768:40960], ls, buf[20480:28672])]
    with pytest.raises(A.AdhaError):
        A.remap_batched(ctx, items)


def test_batched_overlap_check_matches_all_pairs(ctx):
    """Random batches of small items placed in one buffer: the library's
    sorted-sweep check rejects a batch exactly when some item's destination
    overlaps another item's destination or source (all pairs, here)."""
    import random
    rng = random.Random(11)
    st = A.Struct(1000, [A.F32, A.F32, A.F32, A.F32])
    la, ls = A.Layout.aos(st), A.Layout.soa(st)
    na, ns = la.nbytes, ls.nbytes
    slot = 4096
    buf = torch.zeros(64 * slot + ns, dtype=torch.uint8, device="cuda")

    def ov(a, x, b, y):
        return a < b + y and b < a + x

    rejected = 0
    for trial in range(150):
        k = rng.randint(1, 6)
        spans = []
        for _ in range(k):
            s = rng.randrange(64) * slot
            d = rng.randrange(64) * slot
            while ov(s, na, d, ns):
                d = rng.randrange(64) * slot
            spans.append((s, d))
        want = any(ov(spans[i][1], ns, spans[j][1], ns) or ov(spans[i][1], ns, spans[j][0], na) or
                   ov(spans[j][1], ns, spans[i][0], na) for i in range(k) for j in range(i + 1, k))
        items = [(la, buf[s:s + na], ls, buf[d:d + ns]) for s, d in spans]
        if want:
            with pytest.raises(A.AdhaError, match="overlap"):
                A.remap_batched(ctx, items)
            rejected += 1
        else:
            A.remap_batched(ctx, items)
    ctx.check()
    assert 0 < rejected < 150


def test_tuner_picks_a_valid_shape_and_persists(ctx):
    n = (1 << 20) + 77
    spec = synth.config2_struct(n)
    st = A.Struct.from_spec(spec)
    La, Ls = A.Layout.aos(st), A.Layout.soa(st)
    Oa, Os = oaos(n, spec.elem_bytes), OLayout(n, spec.elem_bytes, list(range(16)), [1] * 16)
    cols = synth.record_matrix(2, n, spec.dtypes, spec.elem_bytes)
    src_h = oracle.pack(Oa, cols)
    want = oracle.remap(Oa, src_h, Os)
    src = dev_bytes(src_h)
    dst = torch.empty(Os.nbytes, dtype=torch.uint8, device="cuda")
    res = A.tune_remap(ctx, La, src, Ls, dst, reps=2)
    say("tuned", res)
    assert res["best_us"] <= res["default_us"] * 1.0001
    assert A.get_shape(ctx, La, Ls) == res["shape"]
    dst.fill_(0xA5)
    A.remap(ctx, La, src, Ls, dst)
    ctx.check()
    assert first_diff(host(dst, Os.nbytes), want) is None
    arrs = _arrays(16, 14, seed=7)
    items = [(a["la"], a["src"], a["lb"], a["dst"]) for a in arrs]
    bres = A.tune_batched(ctx, items, reps=2)
    say("tuned batch", bres)
    assert bres["best_us"] <= bres["default_us"] * 1.0001
    A.remap_batched(ctx, items, A.BATCH_GRAPH)
    ctx.check()
    _check(arrs, "tuned batch")
    with tempfile.TemporaryDirectory() as d:
        p = os.path.join(d, "tune.txt")
        A.tune_save(ctx, p)
        ctx2 = A.Ctx(0)
        A.tune_load(ctx2, p)
        # a fresh layout pair of the same class picks the tuned shape up
        st2 = A.Struct.from_spec(spec)
        la2, ls2 = A.Layout.aos(st2), A.Layout.soa(st2)
        got = A.get_shape(ctx2, la2, ls2)
        assert got == res["shape"]
        txt = open(p).read()
        open(p, "w").write(txt.replace("batch", "batcH", 1))
        with pytest.raises(A.AdhaError) as e:
            A.tune_load(ctx2, p)
        assert e.value.status == A.ERR_IO
        with pytest.raises(A.AdhaError):
            A.tune_load(ctx2, os.path.join(d, "missing.txt"))


def _aos_device_array(i, n, eb, seed):
    """AoS buffer of array i drawn on the device: field f of record r holds
    draw r of stream 64*i + f, packed in field order."""
    S = sum(eb)
    t = torch.zeros(max(256, -(-n * S // 256) * 256), dtype=torch.uint8, device="cuda")
    if n == 0:
        return t
    view = t[: n * S].view(n, S)
    off = 0
    for f, e in enumerate(eb):
        z = synth.splitmix64_torch(seed, 64 * i + f, 0, n, "cuda")
        view[:, off:off + e] = synth.decode_torch(z, synth.RAW, e)
        off += e
    return t


@pytest.mark.timeout(900)
def test_config4_full_batch_tuned_policy_matches_oracle(ctx):
    """The whole 512-array batched workload (lengths log-uniform in 2^10 ..
    2^22, 4-24 fields of 4 or 8 bytes, AoS -> SoA or AoSoA): the batch policy
    is tuned as the benchmark tunes it, then the graph launch's output of
    every array is compared byte for byte with the oracle's remap of that
    array, and so is a persistent launch under the default policy of a
    fresh context."""
    arrs = synth.config4_arrays()
    c2 = A.Ctx(0)
    items, keep = [], []
    say("config4 full: drawing", len(arrs), "arrays on the device")
    for i, a in enumerate(arrs):
        eb = a["elem_bytes"]
        st = A.Struct(a["n"], [A.RAW] * len(eb), eb)
        Oa = oaos(a["n"], eb)
        Ob = OLayout(a["n"], eb, a["target_gof"], a["target_tiles"])
        src = _aos_device_array(i, a["n"], eb, 4)
        assert src.numel() >= Oa.nbytes
        dst = torch.full((Ob.nbytes,), 0xA5, dtype=torch.uint8, device="cuda")
        items.append((mirror(st, Oa), src, mirror(st, Ob), dst))
        keep.append((st, Oa, Ob))
    say("config4 full: tuning the batch policy")
    tuned = A.tune_batched(ctx, items, reps=2)
    say("config4 full: tuned", tuned)

    def check(label):
        bad = []
        for i, ((_, Oa, Ob), (_, src, _, dst)) in enumerate(zip(keep, items)):
            want = oracle.remap(Oa, src[: Oa.nbytes].cpu().numpy(), Ob)
            d = first_diff(dst.cpu().numpy(), want)
            if d is not None:
                bad.append((i, d))
        assert not bad, (label, bad[:5])

    for (_, _, _, dst) in items:
        dst.fill_(0xA5)
    say("config4 full: graph launch under the tuned policy")
    A.remap_batched(ctx, items, A.BATCH_GRAPH)
    ctx.check()
    check("tuned graph")
    for (_, _, _, dst) in items:
        dst.fill_(0x5A)
    say("config4 full: persistent launch under the default policy")
    A.remap_batched(c2, items, 0)
    c2.check()
    check("default persistent")
