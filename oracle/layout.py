"""Oracle: the layout address map.  TEST INFRASTRUCTURE ONLY.

The paper (section 1, last paragraph; section 2, first paragraph) considers
AoS and SoA layouts and, through its ODS pass, structures made of clustered
fields; Table 2 gives two such hybrids (AoSU: U1..U3 interleaved, the rest as
separate arrays; AoSV: V1..V3 interleaved) and Table 3 a split of 32 fields
into 4 interleaved structures of 8.  A layout here is therefore a partition
of the struct's fields into groups, each group stored either interleaved
(tile T = 1) or as an array of T-record tiles (AoSoA, T a power of two).

Definition (the readings of what the paper leaves open are listed with the
oracle's other readings):
  * groups are ordered by their smallest field id; inside a group the fields
    are packed in ascending id with no alignment padding;
  * S_g = sum of the element bytes of group g, p_f = byte offset of field f
    inside its group's record;
  * addr(r, f) = base_g + (r div T)*T*S_g + p_f*T + (r mod T)*e_f;
  * B_g = roundup(N, T)*S_g; base_0 = 0, base_{g+1} = roundup(base_g + B_g, 256);
    the layout's size is roundup(base_last + B_last, 256);
  * a one-field group is stored as a plain array, so its tile is taken as 1;
  * every byte not covered by some (r, f) is padding and holds zero.
AoS is one group with T = 1; SoA is one group per field.
"""
from __future__ import annotations

import numpy as np

VALID_ELEM = (1, 2, 4, 8)
GROUP_ALIGN = 256
MAX_TILE = 256
DESC_COLS = 5  # base, tile, group record bytes, offset in record, element bytes


def _roundup(x: int, m: int) -> int:
    return (x + m - 1) // m * m


class Layout:
    """Canonical layout of an N-record struct.

    elem_bytes[f] is e_f; group_of_field[f] is an arbitrary label for f's group;
    tile_of_group[label] is that group's T.
    """

    def __init__(self, n: int, elem_bytes, group_of_field, tile_of_group):
        F = len(elem_bytes)
        if n < 0:
            raise ValueError("n must be >= 0")
        if len(group_of_field) != F:
            raise ValueError("group_of_field needs one label per field")
        for e in elem_bytes:
            if e not in VALID_ELEM:
                raise ValueError(f"element size {e} not in {VALID_ELEM}")
        labels = {}
        for f, g in enumerate(group_of_field):
            labels.setdefault(int(g), []).append(f)
        if sorted(labels) != list(range(len(tile_of_group))):
            raise ValueError("group labels must be exactly 0..n_groups-1")
        groups = []
        for g, fields in labels.items():
            t = int(tile_of_group[g])
            if t < 1 or t > MAX_TILE or (t & (t - 1)):
                raise ValueError(f"tile {t} is not a power of two in [1, {MAX_TILE}]")
            if len(fields) == 1:
                t = 1
            groups.append((tuple(sorted(fields)), t))
        groups.sort(key=lambda gt: gt[0][0])
        self.n = int(n)
        self.elem_bytes = [int(e) for e in elem_bytes]
        self.groups = groups
        self.base, self.S, self.B = [], [], []
        self.group_of = [0] * F
        self.p = [0] * F
        at = 0
        for gi, (fields, t) in enumerate(groups):
            s = 0
            for f in fields:
                self.group_of[f] = gi
                self.p[f] = s
                s += self.elem_bytes[f]
            b = _roundup(self.n, t) * s
            self.base.append(at)
            self.S.append(s)
            self.B.append(b)
            at = _roundup(at + b, GROUP_ALIGN)
        self.nbytes = at

    # -- placement --------------------------------------------------------
    def placed(self, bases) -> "Layout":
        """The same groups at explicit byte offsets (one per group, in group
        order, each a multiple of 256).  Group g then owns the bytes
        [bases[g], bases[g] + roundup(B_g, 256)); regions may not overlap.
        The size is the end of the last region."""
        bases = [int(b) for b in bases]
        if len(bases) != len(self.groups):
            raise ValueError("one base per group is needed")
        ends = []
        for g, b in enumerate(bases):
            if b < 0 or b % GROUP_ALIGN:
                raise ValueError(f"base {b} of group {g} is not a multiple of {GROUP_ALIGN}")
            ends.append(b + _roundup(self.B[g], GROUP_ALIGN))
        spans = sorted((b, e) for b, e in zip(bases, ends) if e > b)
        for (b0, e0), (b1, _) in zip(spans, spans[1:]):
            if b1 < e0:
                raise ValueError("group regions overlap")
        out = Layout.__new__(Layout)
        out.__dict__.update(self.__dict__)
        out.base = bases
        out.nbytes = max(ends) if ends else 0
        return out

    def region(self, g: int):
        """Byte range [start, end) group g owns (its records and padding)."""
        return self.base[g], self.base[g] + _roundup(self.B[g], GROUP_ALIGN)

    # -- identity ---------------------------------------------------------
    def key(self):
        return tuple(self.groups)

    def __eq__(self, other):
        return isinstance(other, Layout) and self.n == other.n and \
            self.elem_bytes == other.elem_bytes and self.key() == other.key()

    def __hash__(self):
        return hash((self.n, tuple(self.elem_bytes), self.key()))

    def __repr__(self):
        return "Layout(" + ", ".join(
            "{" + ",".join(map(str, fs)) + "}" + (f"x{t}" if t > 1 else "")
            for fs, t in self.groups) + ")"

    def tile(self, f: int) -> int:
        return self.groups[self.group_of[f]][1]

    # -- the address map --------------------------------------------------
    def addr(self, r: int, f: int) -> int:
        g = self.group_of[f]
        t = self.groups[g][1]
        return (self.base[g] + (r // t) * t * self.S[g] + self.p[f] * t
                + (r % t) * self.elem_bytes[f])

    def addr_vec(self, r: np.ndarray, f: int) -> np.ndarray:
        r = np.asarray(r, dtype=np.int64)
        g = self.group_of[f]
        t = self.groups[g][1]
        return (self.base[g] + (r // t) * t * self.S[g] + self.p[f] * t
                + (r % t) * self.elem_bytes[f])

    def desc(self) -> np.ndarray:
        """Per-field (base, T, S_g, p_f, e_f) rows, uint64 [F, 5], for the C oracle."""
        d = np.zeros((len(self.elem_bytes), DESC_COLS), np.uint64)
        for f, e in enumerate(self.elem_bytes):
            g = self.group_of[f]
            d[f] = (self.base[g], self.groups[g][1], self.S[g], self.p[f], e)
        return d


def aos(n: int, elem_bytes) -> Layout:
    return Layout(n, elem_bytes, [0] * len(elem_bytes), [1])


def soa(n: int, elem_bytes) -> Layout:
    F = len(elem_bytes)
    return Layout(n, elem_bytes, list(range(F)), [1] * F)


def from_partition(n: int, elem_bytes, parts, tile: int = 1) -> Layout:
    """Layout from a list of field groups (fields not listed become singletons)."""
    F = len(elem_bytes)
    gof = [-1] * F
    labels = 0
    for part in parts:
        for f in part:
            gof[f] = labels
        labels += 1
    tiles = [tile] * labels
    for f in range(F):
        if gof[f] < 0:
            gof[f] = labels
            tiles.append(1)
            labels += 1
    return Layout(n, elem_bytes, gof, tiles)
