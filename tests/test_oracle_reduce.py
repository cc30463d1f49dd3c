"""Pins for the oracle's reduction sections (CPU only)."""
import numpy as np

import oracle
from oracle import reduce as OR
from oracle.layout import Layout, aos, soa, from_partition
from paper_1407_4859_amd import synth

F32, F64, I32 = synth.F32, synth.F64, synth.I32


def _cols_from(values, dtypes):
    out = []
    for v, dt in zip(values, dtypes):
        np_t = {F32: np.float32, F64: np.float64, I32: np.int32}[dt]
        a = np.ascontiguousarray(np.array(v, np_t))
        out.append(a.view(np.uint8).reshape(len(v), a.itemsize))
    return out


def test_hand_example():
    # fields: 0 f32, 1 key (i32), 2 f64, 3 i32; five records, two keys, one bad key
    dtypes = [F32, I32, F64, I32]
    eb = [4, 4, 8, 4]
    vals = [[0.5, 1.25, -2.0, 4.0, 8.0],
            [0, 1, 1, 0, 7],
            [1e16, 1.0, 3.0, -1e16, 2.0],
            [-5, 2_000_000_000, 2_000_000_000, 3, 1]]
    L = aos(5, eb)
    buf = oracle.pack(L, _cols_from(vals, dtypes))
    table, bad = OR.reduce(L, dtypes, [0, 2, 3], 1, 2, buf)
    assert bad == 1
    # key 0: records 0 and 3; key 1: records 1 and 2; record 4 has key 7
    assert table[0] == [4.5, 0.0, -2, 2]          # 1e16 + (-1e16) is exactly 0
    assert table[1] == [-0.75, 4.0, 4_000_000_000, 2]
    # exact rounding: naive left-to-right double sums of 1e16, 1, -1e16 give 0
    L2 = aos(3, [8])
    b2 = oracle.pack(L2, _cols_from([[1e16, 1.0, -1e16]], [F64]))
    t2, _ = OR.reduce(L2, [F64], [0], -1, 1, b2)
    assert t2 == [[1.0, 3]]


def test_generator_values_sum_in_closed_form():
    # the generator's f32 values are m * 2^-23 - 1 with m = z >> 40, so the
    # exact sum is (sum of m) * 2^-23 - n, computed here in integers
    n = 10_000
    z = synth.splitmix64(4, 0, 0, n)
    m = sum(int(x) >> 40 for x in z)
    want = (m - n * (1 << 23)) / float(1 << 23)
    L = soa(n, [4])
    buf = oracle.pack(L, [synth.field_values(4, 0, n, F32)])
    table, bad = OR.reduce(L, [F32], [0], -1, 1, buf)
    assert bad == 0 and table == [[want, n]]
    # int32 values: the exact integer sum
    iv = synth.field_values(4, 1, n, I32).view(np.int32).reshape(-1)
    bi = oracle.pack(L, [synth.field_values(4, 1, n, I32)])
    ti, _ = OR.reduce(L, [I32], [0], -1, 1, bi)
    assert ti == [[sum(int(x) for x in iv), n]]


def test_layout_independence_and_keys():
    n = 1000 + 13
    dtypes = [F32, F64, I32, I32, F32]
    eb = [4, 8, 4, 4, 4]
    cols = synth.record_matrix(5, n, dtypes, eb)
    keys = synth.uniform_index(5, 77, n, 9).astype(np.int32)
    keys[[3, 500]] = [-1, 9]                      # two records with a bad key
    cols[3] = keys.view(np.uint8).reshape(n, 4)
    tables = []
    for L in (aos(n, eb), soa(n, eb), Layout(n, eb, [0] * 5, [64]),
              from_partition(n, eb, [[0, 3], [1, 4]], 1), from_partition(n, eb, [[0, 3, 4]], 8)):
        t, bad = OR.reduce(L, dtypes, [0, 1, 2, 4], 3, 9, oracle.pack(L, cols))
        assert bad == 2
        tables.append(t)
    assert all(t == tables[0] for t in tables)
    assert sum(row[-1] for row in tables[0]) == n - 2
    # by brute force over the records, row by row
    v0 = cols[0].copy().view(np.float32).reshape(-1)
    for k in range(9):
        sel = [r for r in range(n) if keys[r] == k]
        assert tables[0][k][-1] == len(sel)
        assert tables[0][k][0] == sum(float(v0[r]) for r in sel)   # exact: grid of 2^-23


def test_table_cells_encoding():
    table = [[1.5, -3, 7], [-0.0, 5, 0]]
    cells = OR.table_cells(table, [F64, I32], [0, 1])
    assert cells.dtype == np.uint64 and len(cells) == 6
    assert cells[0] == np.array([1.5]).view(np.uint64)[0]
    assert cells[1] == (1 << 64) - 3 and cells[2] == 7
    assert cells[3] == np.array([-0.0]).view(np.uint64)[0] and cells[5] == 0
