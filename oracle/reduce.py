"""Oracle: reduction sections.  TEST INFRASTRUCTURE ONLY.

Section 3 of the paper describes the second K-Means section as a reduction
over all the features of the points (the new cluster centres are sums of
the points that belong to each cluster).  The definition written out here:
for each key k in [0, K), over the records r whose key field holds k (every
record has key 0 when there is no key field),

  table[k][j] = the exact sum of read field j (ascending id) over those
                records -- rounded once to a double for F32 and F64 fields
                (math.fsum rounds the exact sum correctly), an exact Python
                integer for integer fields (I32, U32, U16, U8, I16);
  table[k][n_read] = the number of those records.

Records whose key is outside [0, K) are left out and counted as bad.  The
values are read through the layout's address map, so any layout holding the
same records gives the same table.
"""
from __future__ import annotations

import math

import numpy as np

from .layout import Layout

F32, F64, I32, U32, U8, U16, I16 = 0, 1, 2, 4, 5, 6, 7
INTEGER = {I32: np.int32, U32: np.uint32, U8: np.uint8, U16: np.uint16, I16: np.int16}


def field_values(layout: Layout, buf: np.ndarray, dtype: int, f: int) -> np.ndarray:
    """Values of field f of every record, read at the layout's addresses."""
    r = np.arange(layout.n, dtype=np.int64)
    e = layout.elem_bytes[f]
    a = layout.addr_vec(r, f)
    raw = np.stack([buf[a + b] for b in range(e)], axis=1) if layout.n else np.zeros((0, e), np.uint8)
    raw = np.ascontiguousarray(raw)
    if dtype == F32:
        return raw.view(np.float32).reshape(-1)
    if dtype == F64:
        return raw.view(np.float64).reshape(-1)
    if dtype in INTEGER:
        return raw.view(INTEGER[dtype]).reshape(-1)
    raise ValueError(f"field {f} has no numeric type")


def reduce(layout: Layout, dtypes, read, key: int, n_keys: int, buf: np.ndarray):
    """The reduction table (a list of n_keys rows of len(read) + 1 Python
    numbers) and the number of records with an out-of-range key."""
    read = sorted(read)
    if key >= 0:
        keys = field_values(layout, buf, I32, key).astype(np.int64)
    else:
        keys = np.zeros(layout.n, np.int64)
    bad = int(np.count_nonzero((keys < 0) | (keys >= n_keys)))
    cols = [field_values(layout, buf, dtypes[f], f) for f in read]
    table = []
    for k in range(n_keys):
        sel = keys == k
        row = []
        for f, v in zip(read, cols):
            picked = v[sel]
            if dtypes[f] in INTEGER:
                # int64 holds any sum of fewer than 2^31 such values exactly
                row.append(int(picked.astype(np.int64).sum()))
            else:
                row.append(math.fsum(picked.astype(np.float64).tolist()))
        row.append(int(np.count_nonzero(sel)))
        table.append(row)
    return table, bad


def table_cells(table, dtypes, read) -> np.ndarray:
    """The table as the library stores it: uint64 cells holding IEEE double
    bits for floating-point columns, two's-complement int64 for integer
    columns and counts."""
    read = sorted(read)
    out = []
    for row in table:
        for j, v in enumerate(row):
            if j < len(read) and dtypes[read[j]] not in INTEGER:
                out.append(np.array([v], np.float64).view(np.uint64)[0])
            else:
                out.append(np.uint64(v % (1 << 64)))
    return np.array(out, np.uint64)
