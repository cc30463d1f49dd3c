"""Oracle: the analytic cost model.  TEST INFRASTRUCTURE ONLY.

The paper weights its shortest path with a profile of section times (section
2, third paragraph) and does not say how a profile would be predicted.  The
analytic model below is the "method without the learned part": it prices a
section under a layout by the HBM bytes the layout makes it move.

Effective bytes per record of a section under a layout, with an access
granule g = 128 bytes (the line one random access fetches on the device):
  * streaming access to group G (direct sections, and every write):
    min(S_G, sum over touched fields f of max(e_f, g / T_G));
  * random access to group G (the reads of a gather, per neighbour): an
    interleaved multi-field group costs span + g - 1 where span runs from the
    first to the end of the last touched field of the record; any other
    group costs sum over touched fields of (e_f + g - 1);
  * a gather also reads its 4*d index bytes.
Time = 4 us + N * bytes / (5.6e6 bytes per us); a remap between different
layouts costs 4 us + (bytes of its moving fields, read and written) / 5.6e6,
or 4 us + 2 * N * S / 5.6e6 when the whole struct moves.
Layout classes (for reporting): one interleaved group = AoS; one tiled group
= tiled; only one-field groups = SoA; otherwise tiled if any group is tiled,
else grouped.

The learned model's input features are an encoding chosen by the library,
not a quantity with a definition of its own; the tests pin them against
values worked out by hand, and the network itself is pinned in mlp.py.
"""
from __future__ import annotations

import math

import numpy as np

GRANULE = 128.0
BYTES_PER_US = 5.6e6
LAUNCH_US = 4.0


def _stream_bytes(L, gi, touched):
    fields, T = L.groups[gi]
    b = 0.0
    for f in touched:
        if L.group_of[f] == gi:
            b += max(float(L.elem_bytes[f]), GRANULE / T)
    return min(b, float(L.S[gi]))


def _random_bytes(L, gi, touched):
    fields, T = L.groups[gi]
    mine = [f for f in touched if L.group_of[f] == gi]
    if not mine:
        return 0.0
    if T == 1 and len(fields) > 1:
        lo = min(L.p[f] for f in mine)
        hi = max(L.p[f] + L.elem_bytes[f] for f in mine)
        return (hi - lo) + GRANULE - 1.0
    return sum(L.elem_bytes[f] + GRANULE - 1.0 for f in mine)


def bytes_per_record(read, write, degree, L) -> float:
    b = 0.0
    for gi in range(len(L.groups)):
        if degree == 0:
            b += _stream_bytes(L, gi, read)
        else:
            b += degree * _random_bytes(L, gi, read)
        b += _stream_bytes(L, gi, write)
    if degree:
        b += 4.0 * degree
    return b


def section_us(read, write, degree, L) -> float:
    return LAUNCH_US + L.n * bytes_per_record(read, write, degree, L) / BYTES_PER_US


def remap_us(La, Lb, whole: bool = False) -> float:
    """A remap between different layouts: the bytes of the moving fields
    (planner.remap_bytes) at the model's bandwidth, plus the launch; with
    `whole`, the whole struct moves (an executor that remaps between two
    buffers)."""
    from .planner import remap_bytes
    if La.key() == Lb.key():
        return 0.0
    b = 2.0 * La.n * sum(La.elem_bytes) if whole else float(remap_bytes(La, Lb))
    return LAUNCH_US + b / BYTES_PER_US


def layout_class(L) -> int:
    if len(L.groups) == 1:
        return 0 if L.groups[0][1] == 1 else 2
    if all(len(fs) == 1 for fs, _ in L.groups):
        return 1
    return 2 if any(t > 1 for _, t in L.groups) else 3
