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
