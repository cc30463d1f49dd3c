"""GPU parity of the remap kernels against the oracle (bit-exact)."""
import random

import numpy as np
import pytest
import torch

import oracle
from oracle.layout import Layout as OLayout, aos as oaos, soa as osoa
from paper_1407_4859_amd import adha as A
from paper_1407_4859_amd import synth
from gpu_util import (dev_bytes, dev_empty, fill_aos_device, first_diff, host, host_cores, mirror,
                      oracle_remap_threaded, say)

pytestmark = pytest.mark.gpu


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


def _check_remap(ctx, st, OA, OB, cols, label):
    src_h = oracle.pack(OA, cols)
    want = oracle.remap(OA, src_h, OB)
    src = dev_bytes(src_h)
    dst = dev_empty(OB.nbytes)
    LA, LB = mirror(st, OA), mirror(st, OB)
    say("remap", label, OA, "->", OB, "n", OA.n)
    A.remap(ctx, LA, src, LB, dst)
    ctx.check()
    got = host(dst, OB.nbytes)
    assert first_diff(got, want) is None, (label, first_diff(got, want))
    return LA, LB, src, dst


def test_remap_random_layouts_match_oracle(ctx):
    rng = random.Random(21)
    for trial in range(40):
        F = rng.randint(1, 12)
        byte_mode = trial % 5 == 4
        eb = [rng.choice([1, 2, 4, 8] if byte_mode else [4, 8]) for _ in range(F)]
        n = rng.choice([1, 2, 63, 64, 65, 511, 513, 4097, 30011])
        st = A.Struct(n, [A.RAW] * F, eb)
        OA, OB = _rand_layout(rng, n, eb), _rand_layout(rng, n, eb)
        cols = [synth.field_values(trial, f, n, synth.RAW, e) for f, e in enumerate(eb)]
        _check_remap(ctx, st, OA, OB, cols, f"trial {trial}")


@pytest.mark.parametrize("n", [64 * 512, (1 << 16) + 77])
def test_config2_pairs_small(ctx, n):
    spec = synth.config2_struct(n)
    st = A.Struct.from_spec(spec)
    eb = spec.elem_bytes
    gof, tiles = synth.config2_aosoa()
    cols = synth.record_matrix(2, n, spec.dtypes, eb)
    OA, OS, OT = oaos(n, eb), osoa(n, eb), OLayout(n, eb, gof, tiles)
    for a, b in ((OA, OS), (OS, OA), (OA, OT), (OT, OA), (OS, OT)):
        _check_remap(ctx, st, a, b, cols, "config2")


def test_random_bit_patterns_nan_and_subnormals(ctx):
    n = 5000
    eb = [4] * 8 + [8] * 4
    st = A.Struct(n, [A.F32] * 8 + [A.F64] * 4, eb)
    cols = [synth.field_values(7, f, n, synth.RAW, e) for f, e in enumerate(eb)]
    # plant NaN payloads, -0.0 and subnormals
    cols[0][:4] = np.frombuffer(np.array([0x7FC00001, 0x80000000, 0x00000001, 0xFF800000],
                                         np.uint32).tobytes(), np.uint8).reshape(4, 4)
    cols[8][:2] = np.frombuffer(np.array([0x7FF0000000000001, 0x8000000000000000],
                                         np.uint64).tobytes(), np.uint8).reshape(2, 8)
    _check_remap(ctx, st, oaos(n, eb), osoa(n, eb), cols, "bits")
    _check_remap(ctx, st, osoa(n, eb), OLayout(n, eb, [0] * 6 + [1] * 6, [64, 1]), cols, "bits2")


def test_forced_tile_shapes_agree(ctx):
    n = 20000 + 33
    spec = synth.config3_struct(n)
    st = A.Struct.from_spec(spec)
    eb = spec.elem_bytes
    cols = synth.record_matrix(3, n, spec.dtypes, eb)
    OA = oaos(n, eb)
    OB = OLayout(n, eb, [f // 5 for f in range(32)], [64] * 7)
    src_h = oracle.pack(OA, cols)
    want = oracle.remap(OA, src_h, OB)
    src = dev_bytes(src_h)
    LA, LB = mirror(st, OA), mirror(st, OB)
    for R, K, shift, wg, order, nt in ((64, 8, 6, 4, 1, 1), (128, 8, 5, 2, 2, 1), (64, 4, 31, 8, 2, 2),
                                       (192, 8, 7, 1, 1, 2), (64, 8, 6, 16, 2, 2)):
        say("shape", R, K, shift, wg, order, nt)
        A.set_shape(ctx, LA, LB, R, K, shift, wg, order, nt)
        assert A.get_shape(ctx, LA, LB) == dict(tile_records=R, slots=K, pad_shift=shift, wg_per_cu=wg,
                                                order=order, nontemporal=nt)
        dst = dev_empty(OB.nbytes)
        A.remap(ctx, LA, src, LB, dst)
        ctx.check()
        assert first_diff(host(dst, OB.nbytes), want) is None
    with pytest.raises(A.AdhaError):
        A.set_shape(ctx, LA, LB, 100, 8, 6, 4)        # not a multiple of 64
    with pytest.raises(A.AdhaError):
        A.set_shape(ctx, LA, LB, 1024, 8, 6, 4)       # more chunks than slots


def test_empty_and_invalid(ctx):
    st0 = A.Struct(0, [A.F32, A.F32])
    A.remap(ctx, A.Layout.aos(st0), None, A.Layout.soa(st0), None)
    st = A.Struct(1000, [A.F32, A.I32])
    La, Ls = A.Layout.aos(st), A.Layout.soa(st)
    buf = torch.zeros(1 << 16, dtype=torch.uint8, device="cuda")
    with pytest.raises(A.AdhaError):                     # overlap
        A.remap(ctx, La, buf[:8192], Ls, buf[4096:])
    with pytest.raises(A.AdhaError):                     # capacity
        A.remap(ctx, La, buf[:100], Ls, buf[8192:])
    with pytest.raises(A.AdhaError):                     # misaligned
        A.remap(ctx, La, buf[16:], Ls, buf[16384:])
    other = A.Layout.soa(A.Struct(1000, [A.F32, A.F32]))
    with pytest.raises(A.AdhaError):                     # different struct
        A.remap(ctx, La, buf[:8192], other, buf[16384:])
    ctx.check()


def _config2_full():
    n = 1 << 26
    spec = synth.config2_struct(n)
    st = A.Struct.from_spec(spec)
    eb = spec.elem_bytes
    gof, tiles = synth.config2_aosoa()
    return n, spec, st, oaos(n, eb), osoa(n, eb), OLayout(n, eb, gof, tiles)


def _soa_device(spec, seed, OS):
    """Device buffer in the SoA layout OS holding the seeded values of every
    record (field f's column starts at its group base)."""
    n = spec.n
    t = torch.zeros(OS.nbytes, dtype=torch.uint8, device="cuda")
    chunk = 1 << 24
    for f, (dt, e) in enumerate(zip(spec.dtypes, spec.elem_bytes)):
        base = int(OS.addr_vec(np.array([0]), f)[0])
        col = t[base:base + n * e].view(n, e)
        for s in range(0, n, chunk):
            c = min(chunk, n - s)
            col[s:s + c] = synth.decode_torch(synth.splitmix64_torch(seed, f, s, c, "cuda"), dt, e)
    return t


@pytest.mark.timeout(600)
@pytest.mark.parametrize("target", ["SoA", "AoSoA"])
def test_config2_full_size_from_aos_every_record(ctx, target):
    """AoS -> SoA and AoS -> AoSoA at 2^26 records: the whole destination
    (every record, every padding byte) against the oracle's remap of the
    same input, run over record ranges on the host cores; then the way back
    to AoS against the input."""
    n, spec, st, OA, OS, OT = _config2_full()
    OB = OS if target == "SoA" else OT
    say("config2 full: generating", n, "records in AoS; target", target)
    src = fill_aos_device(spec, 2)
    assert src.numel() == OA.nbytes
    LA, LB = mirror(st, OA), mirror(st, OB)
    dst = dev_empty(OB.nbytes)
    say("config2 full: AoS ->", target, "on the device")
    A.remap(ctx, LA, src, LB, dst)
    ctx.check()
    src_h = src.cpu().numpy()
    say("config2 full: oracle AoS ->", target, "on", host_cores(), "host threads")
    want = oracle_remap_threaded(OA, src_h, OB)
    got = dst.cpu().numpy()
    assert first_diff(got, want) is None, first_diff(got, want)
    del got, want
    say("config2 full:", target, "-> AoS on the device")
    back = dev_empty(OA.nbytes)
    A.remap(ctx, LB, dst, LA, back)
    ctx.check()
    assert torch.equal(back, src)


@pytest.mark.timeout(600)
@pytest.mark.parametrize("source", ["SoA", "AoSoA"])
def test_config2_full_size_to_aos_fresh_input(ctx, source):
    """SoA -> AoS and AoSoA -> AoS at 2^26 records from an input drawn
    directly in the source layout (not produced by the library): every byte
    of the AoS result against the oracle, and against the generator's packed
    record image."""
    n, spec, st, OA, OS, OT = _config2_full()
    OB = OS if source == "SoA" else OT
    say("config2 full: generating", n, "records in", source)
    if source == "SoA":
        src = _soa_device(spec, 2, OS)
    else:
        src_h = oracle_remap_threaded(OA, fill_aos_device(spec, 2).cpu().numpy(), OT)
        src = torch.from_numpy(src_h).cuda()
        del src_h
    LA, LB = mirror(st, OA), mirror(st, OB)
    dst = dev_empty(OA.nbytes)
    say("config2 full:", source, "-> AoS on the device")
    A.remap(ctx, LB, src, LA, dst)
    ctx.check()
    say("config2 full: oracle", source, "-> AoS on", host_cores(), "host threads")
    want = oracle_remap_threaded(OB, src.cpu().numpy(), OA)
    got = dst.cpu().numpy()
    assert first_diff(got, want) is None, first_diff(got, want)
    del got
    packed = fill_aos_device(spec, 2).cpu().numpy()
    assert np.array_equal(packed, want)


# ---------------------------------------------------------------- in-place remaps
def _placed_after(L, Lb, n_extra=0):
    """Lb with the groups it shares with L (same fields and tile) at L's bases
    and its other groups packed after the end of L."""
    at = L.nbytes + 256 * n_extra
    bases = []
    for g, grp in enumerate(Lb.groups):
        if grp in L.groups:
            bases.append(L.base[L.groups.index(grp)])
        else:
            bases.append(at)
            at += -(-Lb.B[g] // 256) * 256
    return Lb.placed(bases)


def test_in_place_remap_random_pairs_match_oracle(ctx):
    """Random pairs of layouts (dword and byte fields, several tiles, ragged
    N): the in-place remap moves only the destination's new groups; the
    whole buffer, untouched bytes included, equals the oracle's."""
    rng = random.Random(31)
    for trial in range(40):
        F = rng.randint(2, 12)
        byte_mode = trial % 4 == 3
        eb = [rng.choice([1, 2, 4, 8] if byte_mode else [4, 8]) for _ in range(F)]
        n = rng.choice([1, 63, 64, 65, 513, 4097, 30011])
        st = A.Struct(n, [A.RAW] * F, eb)
        OA, OB = _rand_layout(rng, n, eb), _rand_layout(rng, n, eb)
        if trial % 3 == 0:      # make them share a group
            OB = OLayout(n, eb, [OA.group_of[f] for f in range(F)], [t for _, t in OA.groups])
            g = rng.randrange(len(OB.groups))
            gof = [OA.group_of[f] if OA.group_of[f] != g else len(OA.groups) for f in range(F)]
            used = {x: i for i, x in enumerate(sorted(set(gof)))}
            OB = OLayout(n, eb, [used[x] for x in gof], [1] * len(used))
        P = _placed_after(OA, OB, n_extra=rng.randint(0, 2))
        cols = [synth.field_values(150 + trial, f, n, synth.RAW, e) for f, e in enumerate(eb)]
        buf_h = np.full(P.nbytes + 512, 0xA5, np.uint8)
        buf_h[: OA.nbytes] = oracle.pack(OA, cols)
        want = oracle.remap_in_place(OA, P, buf_h)
        dev = dev_bytes(buf_h)
        LA = mirror(st, OA)
        LP = mirror(st, OB).place(P.base)
        say("in place", trial, OA, "->", P.base, "n", n)
        A.remap_in_place(ctx, LA, LP, dev)
        ctx.check()
        assert first_diff(host(dev), want) is None, (trial, first_diff(host(dev), want))


def test_in_place_remap_rejects_overlapping_regions(ctx):
    st = A.Struct(1000, [A.F32] * 4)
    La = A.Layout.aos(st)
    Ls = A.Layout.soa(st)
    buf = torch.zeros(1 << 16, dtype=torch.uint8, device="cuda")
    with pytest.raises(A.AdhaError):          # SoA at offset 0 overlaps the AoS record array
        A.remap_in_place(ctx, La, Ls, buf)
    ok = Ls.place([16128 + 4096 * i for i in range(4)])
    A.remap_in_place(ctx, La, ok, buf)
    with pytest.raises(A.AdhaError):          # the buffer is too small for the destination
        A.remap_in_place(ctx, La, ok, buf[:16384])
    ctx.check()


@pytest.mark.timeout(600)
def test_config2_full_size_in_place_partial_remap(ctx):
    """2^26 records in SoA; the target groups fields 0-3 in 64-record tiles
    and keeps fields 4-15 as they are: only fields 0-3 move (2 GiB read and
    written instead of 8 GiB), into space after the SoA arrays.  The whole
    arena against the oracle's in-place remap."""
    n, spec, st, OA, OS, OT = _config2_full()
    eb = spec.elem_bytes
    OB = OLayout(n, eb, [0, 0, 0, 0] + list(range(1, 13)), [64] + [1] * 12)
    P = _placed_after(OS, OB)
    assert P.base[1:] == OS.base[4:]
    say("config2 in place: generating", n, "records in SoA")
    src = _soa_device(spec, 2, OS)
    arena = dev_empty(P.nbytes, fill=0x77)
    arena[: OS.nbytes].copy_(src)
    before = np.full(P.nbytes, 0x77, np.uint8)
    before[: OS.nbytes] = src.cpu().numpy()
    del src
    LS = mirror(st, OS)
    LP = mirror(st, OB).place(P.base)
    A.remap_in_place(ctx, LS, LP, arena)
    ctx.check()
    got = arena.cpu().numpy()
    say("config2 in place: oracle")
    want = oracle.remap_in_place(OS, P, before)
    assert first_diff(got, want) is None, first_diff(got, want)
