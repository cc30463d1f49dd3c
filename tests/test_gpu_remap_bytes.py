"""GPU parity of the remap tile kernel's byte mode (structs with 1- and
2-byte fields) against the oracle, bit-exact: random layouts over several
tiles with a ragged tail, forced tile shapes, a batched launch that mixes
byte and dword structs, and a full-size round trip checked on samples."""
import random

import numpy as np
import pytest
import torch

import oracle
from oracle.layout import Layout as OLayout, aos as oaos, soa as osoa
from paper_1407_4859_amd import adha as A
from paper_1407_4859_amd import synth
from gpu_util import dev_bytes, dev_empty, first_diff, host, mirror, say

pytestmark = pytest.mark.gpu

MIXES = {"8x2B+8x4B": [2] * 8 + [4] * 8, "8x1B+4x2B+4x4B": [1] * 8 + [2] * 4 + [4] * 4,
         "24x1B": [1] * 24, "odd": [1, 2, 8, 1, 4, 2, 1]}


@pytest.fixture(scope="module")
def ctx():
    return A.Ctx(0)


def _rand_layout(rng, n, eb, tiles=(1, 2, 4, 64, 128, 256)):
    F = len(eb)
    ng = rng.randint(1, F)
    gof = [rng.randrange(ng) for _ in range(F)]
    used = {g: i for i, g in enumerate(sorted(set(gof)))}
    gof = [used[g] for g in gof]
    return OLayout(n, eb, gof, [rng.choice(tiles) for _ in used])


def _check(ctx, st, OA, OB, cols, label, want_tiles=True):
    src_h = oracle.pack(OA, cols)
    want = oracle.remap(OA, src_h, OB)
    LA, LB = mirror(st, OA), mirror(st, OB)
    info = A.describe(LA, LB)
    if want_tiles:
        assert info["byte_path"] == 1 and info["full_tiles"] >= 2, (label, info)
    dst = dev_empty(OB.nbytes)
    say("byte remap", label, OA, "->", OB, "n", OA.n, "tiles", info["full_tiles"])
    A.remap(ctx, LA, dev_bytes(src_h), LB, dst)
    ctx.check()
    d = first_diff(host(dst, OB.nbytes), want)
    assert d is None, (label, d)


def test_random_sub_dword_layouts(ctx):
    rng = random.Random(31)
    for trial in range(36):
        F = rng.randint(1, 14)
        eb = [rng.choice([1, 2, 4, 8]) for _ in range(F)]
        if all(e >= 4 for e in eb):
            eb[rng.randrange(F)] = rng.choice([1, 2])
        S = sum(eb)
        # several tiles of up to 16 KiB plus a ragged tail
        n = rng.choice([3, 5, 9]) * max(256, 16384 // S) + rng.randint(1, 255)
        st = A.Struct(n, [A.RAW] * F, eb)
        OA, OB = _rand_layout(rng, n, eb), _rand_layout(rng, n, eb)
        cols = [synth.field_values(100 + trial, f, n, synth.RAW, e) for f, e in enumerate(eb)]
        _check(ctx, st, OA, OB, cols, f"trial {trial}")


@pytest.mark.parametrize("mix", sorted(MIXES))
def test_aos_soa_tiled_pairs(ctx, mix):
    eb = MIXES[mix]
    n = 40 * 1024 + 77
    st = A.Struct(n, [A.RAW] * len(eb), eb)
    cols = [synth.field_values(7, f, n, synth.RAW, e) for f, e in enumerate(eb)]
    F = len(eb)
    OA, OS = oaos(n, eb), osoa(n, eb)
    OT = OLayout(n, eb, [0] * F, [64])
    OG = OLayout(n, eb, [f % 3 for f in range(F)], [1, 4, 128][: min(3, F)])
    for a, b in ((OA, OS), (OS, OA), (OA, OT), (OT, OS), (OG, OA), (OS, OG)):
        _check(ctx, st, a, b, cols, mix)


def test_forced_shapes_in_byte_mode(ctx):
    eb = MIXES["8x1B+4x2B+4x4B"]
    n = 20000 + 33
    st = A.Struct(n, [A.RAW] * len(eb), eb)
    cols = [synth.field_values(5, f, n, synth.RAW, e) for f, e in enumerate(eb)]
    OA = oaos(n, eb)
    OB = OLayout(n, eb, [f // 5 for f in range(len(eb))], [64, 1, 128, 4])
    src_h = oracle.pack(OA, cols)
    want = oracle.remap(OA, src_h, OB)
    src = dev_bytes(src_h)
    LA, LB = mirror(st, OA), mirror(st, OB)
    for R, K, shift, wg, order, nt in ((128, 1, 6, 4, 1, 1), (256, 2, 5, 2, 2, 1), (512, 4, 31, 8, 2, 2),
                                       (1024, 8, 7, 1, 1, 2), (384, 4, 2, 16, 2, 2)):
        say("byte shape", R, K, shift, wg, order, nt)
        A.set_shape(ctx, LA, LB, R, K, shift, wg, order, nt)
        dst = dev_empty(OB.nbytes)
        A.remap(ctx, LA, src, LB, dst)
        ctx.check()
        assert first_diff(host(dst, OB.nbytes), want) is None, (R, K, shift)
    with pytest.raises(A.AdhaError):
        A.set_shape(ctx, LA, LB, 64, 4, 6, 4)            # not a multiple of the 128-record tile
    A.set_shape(ctx, LA, LB)                               # back to automatic


def test_batched_mixes_byte_and_dword_structs(ctx):
    """One persistent launch in byte mode over arrays of both kinds."""
    rng = random.Random(9)
    arrs = []
    for i in range(12):
        F = rng.randint(2, 10)
        eb = [rng.choice([1, 2, 4, 8] if i % 2 else [4, 8]) for _ in range(F)]
        n = rng.randint(2000, 60000)
        st = A.Struct(n, [A.RAW] * F, eb)
        OA, OB = _rand_layout(rng, n, eb), _rand_layout(rng, n, eb)
        cols = [synth.field_values(40 + i, f, n, synth.RAW, e) for f, e in enumerate(eb)]
        src_h = oracle.pack(OA, cols)
        arrs.append(dict(la=mirror(st, OA), lb=mirror(st, OB), src=dev_bytes(src_h), OB=OB,
                         want=oracle.remap(OA, src_h, OB),
                         dst=torch.full((OB.nbytes,), 0xA5, dtype=torch.uint8, device="cuda")))
    say("byte batched", len(arrs))
    batch = A.BatchItems([(a["la"], a["src"], a["lb"], a["dst"]) for a in arrs])
    A.remap_batched(ctx, batch, 0)
    ctx.check()
    for i, a in enumerate(arrs):
        assert first_diff(host(a["dst"], a["OB"].nbytes), a["want"]) is None, i
    for rep in range(2):                    # graph replays, with eager work between them
        for a in arrs:
            a["dst"].fill_(0x3C)
        torch.cuda.synchronize()
        say("byte batched graph replay", rep)
        A.remap_batched(ctx, batch, A.BATCH_GRAPH)
        ctx.check()
        for i, a in enumerate(arrs):
            assert first_diff(host(a["dst"], a["OB"].nbytes), a["want"]) is None, (rep, i)


@pytest.mark.timeout(600)
def test_full_size_round_trip_sampled(ctx):
    """2^25 records of 8 one-byte, 4 two-byte and 4 four-byte fields:
    AoS -> SoA and AoS -> grouped-tiled checked on sampled records against
    the generator, then back to AoS byte for byte."""
    n = 1 << 25
    eb = MIXES["8x1B+4x2B+4x4B"]
    F, S = len(eb), sum(eb)
    st = A.Struct(n, [A.RAW] * F, eb)
    OA, OS = oaos(n, eb), osoa(n, eb)
    OG = OLayout(n, eb, [f % 3 for f in range(F)], [1, 4, 128])
    say("byte full: generating", n, "records")
    src = torch.zeros(OA.nbytes, dtype=torch.uint8, device="cuda")
    view = src[: n * S].view(n, S)
    offs = np.concatenate([[0], np.cumsum(eb)[:-1]])
    chunk = 1 << 24
    for f, e in enumerate(eb):
        for s0 in range(0, n, chunk):
            z = synth.splitmix64_torch(11, f, s0, chunk, "cuda")
            view[s0:s0 + chunk, offs[f]:offs[f] + e] = synth.decode_torch(z, synth.RAW, e)
    rng = np.random.default_rng(1)
    recs = np.unique(np.concatenate([rng.integers(0, n, 300), [0, 1, n - 1, n - 640, n // 2]]))
    back = torch.empty(OA.nbytes, dtype=torch.uint8, device="cuda")
    for OB in (OS, OG):
        LA, LB = mirror(st, OA), mirror(st, OB)
        assert A.describe(LA, LB)["byte_path"] == 1
        dst = torch.empty(OB.nbytes, dtype=torch.uint8, device="cuda")
        say("byte full: AoS ->", OB)
        A.remap(ctx, LA, src, LB, dst)
        ctx.check()
        for f, e in enumerate(eb):
            want = synth.field_values_at(11, f, recs, synth.RAW, e)
            addr = torch.from_numpy(OB.addr_vec(recs, f)).cuda()
            got = torch.stack([dst[addr + k] for k in range(e)], 1).cpu().numpy()
            assert np.array_equal(got, want), (OB, f)
        A.remap(ctx, LB, dst, LA, back)
        ctx.check()
        assert torch.equal(back, src), OB
