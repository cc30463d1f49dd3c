"""Pins for the oracle's layout address map (CPU only)."""
import os
import random

import numpy as np
import pytest

from oracle import layout as OL
from oracle.layout import Layout, aos, soa, from_partition

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _roundup(x, m):
    return -(-x // m) * m


@pytest.mark.parametrize("n", [0, 1, 5, 64, 100])
def test_aos_closed_form(n):
    eb = [4, 8, 2, 1, 4]
    L = aos(n, eb)
    S = sum(eb)
    for r in range(n):
        off = 0
        for f, e in enumerate(eb):
            assert L.addr(r, f) == r * S + off
            off += e
    assert L.nbytes == _roundup(n * S, 256)


@pytest.mark.parametrize("n", [0, 1, 7, 256, 300])
def test_soa_closed_form(n):
    eb = [4, 8, 4, 1]
    L = soa(n, eb)
    base = 0
    for f, e in enumerate(eb):
        for r in range(n):
            assert L.addr(r, f) == base + r * e
        base += _roundup(n * e, 256)
    assert L.nbytes == base


@pytest.mark.parametrize("T", [2, 4, 64])
def test_aosoa_matches_numpy_transpose(T):
    # AoSoA of one group with uniform 4-byte fields is the AoS matrix cut into
    # T-record blocks, each block transposed to field-major.
    n, F = 4 * T, 5
    A = np.arange(n * F, dtype=np.uint32).reshape(n, F)
    L = Layout(n, [4] * F, [0] * F, [T])
    expect = np.ascontiguousarray(A.reshape(n // T, T, F).transpose(0, 2, 1)).reshape(-1)
    img = np.zeros(L.nbytes // 4, np.uint32)
    for r in range(n):
        for f in range(F):
            img[L.addr(r, f) // 4] = A[r, f]
    assert np.array_equal(img[: n * F], expect)


def _random_layout(rng, n, eb):
    F = len(eb)
    ng = rng.randint(1, F)
    gof = [rng.randrange(ng) for _ in range(F)]
    used = sorted(set(gof))
    remap = {g: i for i, g in enumerate(used)}
    gof = [remap[g] for g in gof]
    tiles = [rng.choice([1, 2, 4, 8, 64]) for _ in used]
    return Layout(n, eb, gof, tiles)


def test_bijective_and_in_bounds():
    rng = random.Random(7)
    for _ in range(60):
        F = rng.randint(1, 8)
        eb = [rng.choice([1, 2, 4, 8]) for _ in range(F)]
        n = rng.randint(0, 300)
        L = _random_layout(rng, n, eb)
        owner = np.full(L.nbytes, -1, np.int64)
        for f, e in enumerate(eb):
            a = L.addr_vec(np.arange(n), f)
            for b in range(e):
                assert np.all(owner[a + b] == -1), "two elements share a byte"
                owner[a + b] = f
        for b in L.base:
            assert b % 256 == 0
        # elements of a record inside one group are contiguous when T == 1
        for fields, t in L.groups:
            if t == 1 and n > 0:
                addrs = [L.addr(n - 1, f) for f in fields]
                assert addrs == sorted(addrs)


def test_canonical_form():
    eb = [4, 4, 4]
    # labels are arbitrary; groups get ordered by smallest field id
    a = Layout(10, eb, [1, 0, 1], [1, 1])
    b = Layout(10, eb, [0, 1, 0], [1, 1])
    assert a == b and a.groups[0][0] == (0, 2)
    # a lone field is stored as a plain array whatever tile it was given
    c = Layout(10, eb, [0, 1, 2], [64, 1, 8])
    assert c == soa(10, eb)
    for bad in ([3], [0], [1000]):
        with pytest.raises(ValueError):
            Layout(10, eb, [0, 0, 0], bad if bad != [1000] else [512])
    with pytest.raises(ValueError):
        Layout(10, [3, 4, 4], [0, 0, 0], [1])
    with pytest.raises(ValueError):
        Layout(10, eb, [0, 2, 2], [1, 1, 1])  # label 1 unused


def _parse_table2():
    names, rows = None, {}
    with open(os.path.join(GOLDEN, "table2_medical_layouts.txt")) as fh:
        for line in fh:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            key, spec = line.split(":", 1)
            groups, cur, inside = [], "", False
            order = []
            for tok in spec.replace(" ", "").split(","):
                if tok.startswith("{"):
                    inside, cur = True, [tok[1:]]
                    if tok.endswith("}"):
                        inside = False
                        cur[-1] = cur[-1][:-1]
                        groups.append(cur)
                elif inside:
                    if tok.endswith("}"):
                        cur.append(tok[:-1])
                        groups.append(cur)
                        inside = False
                    else:
                        cur.append(tok)
                else:
                    groups.append([tok])
            order = [nm for g in groups for nm in g]
            if names is None:
                names = order
            rows[key] = groups
    return names, rows


def test_table2_layouts_encode():
    names, rows = _parse_table2()
    assert len(names) == 9 and set(rows) == {"SoA", "AoSU", "AoSV"}
    ids = {nm: i for i, nm in enumerate(names)}
    n, eb = 100, [4] * 9
    lay = {}
    for key, groups in rows.items():
        parts = [[ids[nm] for nm in g] for g in groups if len(g) > 1]
        lay[key] = from_partition(n, eb, parts, 1)
    assert lay["SoA"] == soa(n, eb)
    for key, trio in (("AoSU", ["U1", "U2", "U3"]), ("AoSV", ["V1", "V2", "V3"])):
        L = lay[key]
        multi = [fs for fs, t in L.groups if len(fs) > 1]
        assert multi == [tuple(ids[nm] for nm in trio)]
        # the trio is interleaved: 12-byte records, fields at +0, +4, +8
        for r in (0, 1, 57):
            a0 = L.addr(r, ids[trio[0]])
            assert [L.addr(r, ids[nm]) - a0 for nm in trio] == [0, 4, 8]
            assert L.addr(r + 1, ids[trio[0]]) - a0 == 12
        # every other field is a plain array
        for nm in names:
            if nm not in trio:
                assert L.addr(1, ids[nm]) - L.addr(0, ids[nm]) == 4
