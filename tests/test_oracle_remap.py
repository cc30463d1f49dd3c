"""Pins for the oracle's remap (CPU only)."""
import random

import numpy as np
import pytest

import oracle
from oracle.layout import Layout, aos, soa
from paper_1407_4859_amd import synth


def _rand_cols(seed, n, eb):
    return [synth.field_values(seed, f, n, synth.RAW, e) for f, e in enumerate(eb)]


@pytest.mark.parametrize("n", [64, 4096])
def test_aos_to_soa_is_numpy_transpose(n):
    F = 16
    eb = [4] * F
    A = synth.splitmix64(2, 0, 0, n * F).astype(np.uint32).reshape(n, F)  # raw bit patterns
    src = A.view(np.uint8).reshape(-1).copy()
    out = oracle.remap(aos(n, eb), src, soa(n, eb))
    expect = np.ascontiguousarray(A.T).view(np.uint8).reshape(-1)
    assert np.array_equal(out, expect)
    back = oracle.remap(soa(n, eb), out, aos(n, eb))
    assert np.array_equal(back, src)


def test_aos_to_aosoa_is_blocked_transpose():
    n, T = 256, 64
    gof, tiles = synth.config2_aosoa()
    eb = [4] * 16
    A = np.arange(n * 16, dtype=np.uint32).reshape(n, 16)
    src = A.view(np.uint8).reshape(-1).copy()
    Ld = Layout(n, eb, gof, tiles)
    out = oracle.remap(aos(n, eb), src, Ld).view(np.uint32)
    # groups {0-3}, {4-7}, {8-15}: each is its own block-transposed array
    at = 0
    for lo, hi in ((0, 4), (4, 8), (8, 16)):
        blk = A[:, lo:hi].reshape(n // T, T, hi - lo).transpose(0, 2, 1).reshape(-1)
        assert np.array_equal(out[at:at + blk.size], blk)
        at += blk.size


def _rand_layout(rng, n, eb):
    F = len(eb)
    ng = rng.randint(1, F)
    gof = [rng.randrange(ng) for _ in range(F)]
    used = {g: i for i, g in enumerate(sorted(set(gof)))}
    gof = [used[g] for g in gof]
    return Layout(n, eb, gof, [rng.choice([1, 4, 64, 128]) for _ in used])


def test_round_trip_and_composition():
    rng = random.Random(11)
    for trial in range(40):
        F = rng.randint(1, 10)
        eb = [rng.choice([1, 2, 4, 8]) for _ in range(F)]
        n = rng.choice([0, 1, 2, 63, 64, 65, rng.randint(1, 700)])
        L0, L1, L2 = (_rand_layout(rng, n, eb) for _ in range(3))
        cols = _rand_cols(trial % 200, n, eb)
        b0 = oracle.pack(L0, cols)
        b1 = oracle.remap(L0, b0, L1)
        assert np.array_equal(oracle.remap(L1, b1, L0), b0)          # inverse
        direct = oracle.remap(L0, b0, L2)
        assert np.array_equal(oracle.remap(L1, b1, L2), direct)      # composition
        for f in range(F):                                           # values preserved
            assert np.array_equal(oracle.unpack(L2, direct, f), cols[f])
        assert not direct[oracle.padding_mask(L2)].any()             # padding zero


def test_range_split_equals_whole():
    n, eb = 1000, [4, 8, 4]
    cols = _rand_cols(5, n, eb)
    L0 = aos(n, eb)
    L1 = Layout(n, eb, [0, 0, 1], [64, 1])
    b0 = oracle.pack(L0, cols)
    whole = oracle.remap(L0, b0, L1)
    part = np.zeros(L1.nbytes, np.uint8)
    for lo in range(0, n, 333):
        oracle.remap(L0, b0, L1, lo, min(n, lo + 333), out=part)
    assert np.array_equal(part, whole)


# ---------------------------------------------------------------- moving fields
def test_table2_moving_fields_match_the_hand_worked_list():
    """The oracle's moving-field rule against the moving sets worked out by
    hand for the remaps between Table 2's Medical layouts."""
    import os
    from oracle.planner import moving_fields, remap_bytes
    from test_oracle_layout import GOLDEN, _parse_table2
    from oracle.layout import from_partition
    names, rows = _parse_table2()
    ids = {nm: i for i, nm in enumerate(names)}
    n, eb = 1000, [4] * 9
    lay = {k: from_partition(n, eb, [[ids[nm] for nm in g] for g in groups if len(g) > 1], 1)
           for k, groups in rows.items()}
    seen = 0
    with open(os.path.join(GOLDEN, "table2_remap_fields.txt")) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            pair, moved = line.split(":", 1)
            a, b = (x.strip() for x in pair.split("->"))
            want = {nm for nm in moved.replace(" ", "").split(",") if nm}
            got = {names[f] for f in moving_fields(lay[a], lay[b])}
            assert got == want, (a, b, got, want)
            assert remap_bytes(lay[a], lay[b]) == 2 * n * 4 * len(want)
            seen += 1
    assert seen == 7


def test_moving_fields_special_cases():
    """AoS <-> SoA moves every field (the whole-struct remap, 2*N*S bytes);
    equal layouts move nothing; a change of tile alone moves that group."""
    from oracle.planner import moving_fields, remap_bytes
    n, eb = 777, [4, 8, 4, 2, 1, 4]
    A, S = aos(n, eb), soa(n, eb)
    assert moving_fields(A, S) == list(range(6)) and remap_bytes(A, S) == 2 * n * sum(eb)
    assert moving_fields(S, S) == [] and remap_bytes(A, A) == 0
    L1 = Layout(n, eb, [0, 0, 1, 2, 2, 3], [1, 1, 1, 1])
    L2 = Layout(n, eb, [0, 0, 1, 2, 2, 3], [64, 1, 1, 1])   # group {0,1} tiled by 64
    assert moving_fields(L1, L2) == [0, 1]
    L3 = Layout(n, eb, [0, 0, 1, 1, 2, 3], [1, 1, 1, 1])    # field 3 joins field 2
    assert moving_fields(L1, L3) == [2, 3, 4]
    assert remap_bytes(L1, L3) == 2 * n * (4 + 2 + 1)
    # a singleton keeps its placement whatever its nominal tile
    assert moving_fields(Layout(n, eb, [0, 0, 1, 2, 2, 3], [1, 64, 1, 1]), L1) == []


# ---------------------------------------------------------------- in-place remap
def _placed_after(L, Lb, n_extra=0):
    """Lb with the groups it shares with L (same fields and tile) at L's
    bases and its other groups packed after the end of L."""
    at = L.nbytes + 256 * n_extra
    bases = []
    for g, grp in enumerate(Lb.groups):
        if grp in L.groups:
            bases.append(L.base[L.groups.index(grp)])
        else:
            bases.append(at)
            at += -(-Lb.B[g] // 256) * 256
    return Lb.placed(bases)


def _rand_layout(rng, n, eb):
    F = len(eb)
    ng = rng.randint(1, F)
    gof = [rng.randrange(ng) for _ in range(F)]
    used = {g: i for i, g in enumerate(sorted(set(gof)))}
    return Layout(n, eb, [used[g] for g in gof], [rng.choice([1, 2, 4, 64]) for _ in used])


def test_in_place_remap_into_fresh_space_is_the_plain_remap():
    """With no group in common the in-place remap writes the whole struct
    after the source: those bytes are the plain remap's result, shifted, and
    the source bytes are untouched."""
    rng = random.Random(3)
    for trial in range(12):
        F = rng.randint(1, 7)
        eb = [rng.choice([1, 2, 4, 8]) for _ in range(F)]
        n = rng.choice([1, 5, 64, 333])
        La, Lb = aos(n, eb), soa(n, eb)
        src = oracle.pack(La, _rand_cols(trial, n, eb))
        buf = np.concatenate([src, np.full(Lb.nbytes + 512, 0xC3, np.uint8)])
        # every group at a new base (even a group both layouts share moves
        # when its base changes)
        P = Lb.placed([b + La.nbytes for b in Lb.base])
        out = oracle.remap_in_place(La, P, buf)
        assert np.array_equal(out[: La.nbytes], src)
        assert np.array_equal(out[La.nbytes: La.nbytes + Lb.nbytes], oracle.remap(La, src, Lb))
        assert np.array_equal(out[La.nbytes + Lb.nbytes:], buf[La.nbytes + Lb.nbytes:])


def test_in_place_remap_leaves_every_other_byte_and_round_trips():
    """Random pairs of layouts: only the regions of the destination's new
    groups change, the values land at the destination layout's addresses,
    and moving back to the source placement restores the source regions."""
    rng = random.Random(5)
    for trial in range(40):
        F = rng.randint(2, 9)
        eb = [rng.choice([1, 2, 4, 8]) for _ in range(F)]
        n = rng.choice([1, 63, 64, 65, 200])
        La, Lb = _rand_layout(rng, n, eb), _rand_layout(rng, n, eb)
        cols = _rand_cols(100 + trial, n, eb)
        src = oracle.pack(La, cols)
        P = _placed_after(La, Lb, n_extra=rng.randint(0, 2))
        buf = np.concatenate([src, np.full(P.nbytes - La.nbytes + 300, 0x5A, np.uint8)])
        out = oracle.remap_in_place(La, P, buf)
        # the values sit at P's addresses
        for f in range(F):
            assert np.array_equal(oracle.unpack(P, out, f), cols[f]), (trial, f)
        # only the regions of the groups P does not share with La changed
        changed = np.zeros(buf.size, bool)
        for g, grp in enumerate(P.groups):
            if grp not in La.groups:
                a, b = P.region(g)
                changed[a:b] = True
        assert np.array_equal(out[~changed], buf[~changed])
        # padding inside the moved regions is zero
        pad = oracle.padding_mask(P)
        assert not out[: P.nbytes][pad & changed[: P.nbytes]].any()
        # and back: the source regions hold the source bytes again
        back = oracle.remap_in_place(P, La, out)
        assert np.array_equal(back[: La.nbytes], src), trial


def test_in_place_composition():
    """L -> L' -> L'' in place gives the values L -> L'' gives directly."""
    rng = random.Random(9)
    for trial in range(15):
        F = rng.randint(2, 8)
        eb = [rng.choice([4, 8]) for _ in range(F)]
        n = rng.choice([64, 129])
        L0, L1, L2 = (_rand_layout(rng, n, eb) for _ in range(3))
        cols = _rand_cols(200 + trial, n, eb)
        src = oracle.pack(L0, cols)
        P1 = _placed_after(L0, L1)
        # L2 after both: its groups shared with L1 stay where P1 put them
        at = P1.nbytes
        bases = []
        for g, grp in enumerate(L2.groups):
            if grp in P1.groups:
                bases.append(P1.base[P1.groups.index(grp)])
            else:
                bases.append(at)
                at += -(-L2.B[g] // 256) * 256
        P2 = L2.placed(bases)
        buf = np.zeros(max(P1.nbytes, P2.nbytes) + 256, np.uint8)
        buf[: src.size] = src
        two = oracle.remap_in_place(P1, P2, oracle.remap_in_place(L0, P1, buf))
        for f in range(F):
            assert np.array_equal(oracle.unpack(P2, two, f), cols[f]), (trial, f)
