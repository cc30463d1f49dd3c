"""Oracle: the analytic cost model and the cost-model features.  TEST
INFRASTRUCTURE ONLY.

The paper weights its shortest path with a profile of section times (section
2, third paragraph) and does not say how a profile would be predicted.  The
analytic model below is the "method without the learned part": it prices a
section under a layout by the HBM bytes the layout makes it move.

Effective bytes per record of a section under a layout, with a DRAM access
granule g = 64 bytes:
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

Features (16 values, float32, fixed scaling), describing the section and
the groups it touches:
  log2 N / 24, |R| / 16, |W| / 2, d / 32, log2(1 + read bytes) / 8,
  log2(1 + write bytes) / 8, groups holding R / 16, groups holding W / 2,
  whether a gather's reads share one interleaved group spanning <= 64 bytes
  (fetched whole per neighbour), those wide loads per neighbour / 16,
  shares of the read fields in one-field groups, in interleaved groups of
  several fields and in tiled groups of several fields, share of the write
  fields in groups of several fields, for gathers log2(N * record bytes of
  the groups holding R) / 32 (0 for direct sections), log2(effective
  bytes) / 12.
The learned model predicts ln(measured time / section_us), a correction of
the analytic estimate.
Layout classes (for reporting): one interleaved group = AoS; one tiled group
= tiled; only one-field groups = SoA; otherwise tiled if any group is tiled,
else grouped.
"""
from __future__ import annotations

import math

import numpy as np

GRANULE = 64.0
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


def span_loads(read, degree, L) -> int:
    """Wide loads per neighbour of a gather whose reads all sit in one
    interleaved group spanning at most 64 bytes (A-byte loads, A the largest
    of 16, 8, 4 dividing the group record); 0 when that does not apply."""
    if degree == 0 or not read:
        return 0
    groups = {L.group_of[f] for f in read}
    if len(groups) != 1:
        return 0
    g = groups.pop()
    if L.groups[g][1] != 1:
        return 0
    S = L.S[g]
    lo = min(L.p[f] for f in read)
    hi = max(L.p[f] + L.elem_bytes[f] for f in read)
    A = 16 if S % 16 == 0 else 8 if S % 8 == 0 else 4
    lo_a = lo // A * A
    nvec = -(-(hi - lo_a) // A)
    return 0 if nvec * A // 4 > 16 else nvec


def features(read, write, degree, L, spec=None):
    eb = L.elem_bytes
    rb = sum(eb[f] for f in read)
    wb = sum(eb[f] for f in write)
    rg = {L.group_of[f] for f in read}
    wg = {L.group_of[f] for f in write}

    def kind(f):
        fields, T = L.groups[L.group_of[f]]
        return 0 if len(fields) == 1 else (1 if T == 1 else 2)

    kr = [kind(f) for f in read]
    nr, nw = max(1, len(read)), max(1, len(write))
    foot = float(sum(L.S[g] for g in rg)) * L.n
    sl = span_loads(read, degree, L)
    v = [math.log2(max(1, L.n)) / 24.0, len(read) / 16.0, len(write) / 2.0, degree / 32.0,
         math.log2(1.0 + rb) / 8.0, math.log2(1.0 + wb) / 8.0,
         len(rg) / 16.0, len(wg) / 2.0, float(sl > 0), sl / 16.0,
         kr.count(0) / nr, kr.count(1) / nr, kr.count(2) / nr,
         sum(1 for f in write if kind(f) != 0) / nw,
         math.log2(max(1.0, foot)) / 32.0 if degree else 0.0,
         math.log2(max(1.0, bytes_per_record(read, write, degree, L))) / 12.0]
    return np.array(v, np.float64).astype(np.float32)
