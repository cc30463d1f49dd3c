"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle tests.

This module holds no part of the layout method: it only draws numbers.  Every
value comes from one counter-based generator, SplitMix64 (Steele, Lea and
Flood, "Fast splittable pseudorandom number generators", OOPSLA 2014): the
i-th draw of stream ``s`` under seed ``k`` is

    z = mix64(((k << 56) | (s << 36)) + i + 1) * GAMMA)          (mod 2^64)

i.e. the published SplitMix64 sequence started from state
``((k << 56) | (s << 36)) * GAMMA``.  Two implementations are given, numpy
(host) and torch int64 (device, used only to fill large buffers quickly);
tests check that they agree.

Field values are decoded from z as follows, all exactly representable:
  fp32 U[-1,1):  (z >> 40) * 2^-23 - 1
  fp64 U[-1,1):  (z >> 11) * 2^-52 - 1
  int32 U[0,2^31): z >> 33
  raw 32 / 64 bit: low 32 bits of z / z itself (any bit pattern: NaN, -0, subnormal)
  index U[0,n):  ((z >> 32) * n) >> 32      (multiply-shift)
"""
from __future__ import annotations

import numpy as np

GAMMA = 0x9E3779B97F4A7C15
M1 = 0xBF58476D1CE4E5B9
M2 = 0x94D049BB133111EB
MASK64 = (1 << 64) - 1

# dtype codes (same numbering as the C-ABI's adha_dtype)
F32, F64, I32, RAW, U32, U8, U16, I16 = 0, 1, 2, 3, 4, 5, 6, 7
DT_NAMES = {F32: "f32", F64: "f64", I32: "i32", RAW: "raw", U32: "u32", U8: "u8", U16: "u16", I16: "i16"}


def _key(seed: int, stream: int) -> int:
    if not (0 <= seed < 256 and 0 <= stream < (1 << 20)):
        raise ValueError("seed must be < 256 and stream < 2^20")
    return (seed << 56) | (stream << 36)


# ---------------------------------------------------------------- numpy side
def splitmix64(seed: int, stream: int, start: int, count: int) -> np.ndarray:
    """Draws start..start+count-1 of (seed, stream) as uint64."""
    return splitmix64_at(seed, stream, np.arange(start, start + count, dtype=np.uint64))


def splitmix64_at(seed: int, stream: int, counters) -> np.ndarray:
    """Draws number counters[k] of (seed, stream), for any counters, as uint64."""
    with np.errstate(over="ignore"):
        i = np.asarray(counters, dtype=np.uint64) + np.uint64(1)
        z = (np.uint64(_key(seed, stream)) + i) * np.uint64(GAMMA)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(M1)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(M2)
        return z ^ (z >> np.uint64(31))


def splitmix64_scalar(seed: int, stream: int, i: int) -> int:
    """Plain-integer form of the same draw (used to check the vector forms)."""
    z = ((_key(seed, stream) + i + 1) * GAMMA) & MASK64
    z = ((z ^ (z >> 30)) * M1) & MASK64
    z = ((z ^ (z >> 27)) * M2) & MASK64
    return z ^ (z >> 31)


def decode(z: np.ndarray, dtype: int, elem_bytes: int = 4) -> np.ndarray:
    """Decode uint64 draws into raw little-endian element bytes (uint8 [n, e])."""
    if dtype == F32:
        v = ((z >> np.uint64(40)).astype(np.float64) * 2.0 ** -23 - 1.0).astype(np.float32)
    elif dtype == F64:
        v = (z >> np.uint64(11)).astype(np.float64) * 2.0 ** -52 - 1.0
    elif dtype == I32:
        v = (z >> np.uint64(33)).astype(np.int32)
    elif dtype == U32:
        v = (z >> np.uint64(32)).astype(np.uint32)
    elif dtype == U16:
        v = (z >> np.uint64(48)).astype(np.uint16)
    elif dtype == I16:
        v = (z >> np.uint64(48)).astype(np.uint16).view(np.int16)
    elif dtype == U8:
        v = (z >> np.uint64(56)).astype(np.uint8)
    elif dtype == RAW:
        if elem_bytes == 8:
            v = z.copy()
        elif elem_bytes == 4:
            v = (z & np.uint64(0xFFFFFFFF)).astype(np.uint32)
        elif elem_bytes == 2:
            v = (z & np.uint64(0xFFFF)).astype(np.uint16)
        elif elem_bytes == 1:
            v = (z & np.uint64(0xFF)).astype(np.uint8)
        else:
            raise ValueError(elem_bytes)
    else:
        raise ValueError(dtype)
    return np.ascontiguousarray(v).view(np.uint8).reshape(len(z), v.dtype.itemsize)


def decode_wide(z: np.ndarray, dtype: int, lo_exp: int = -40, hi_exp: int = 40) -> np.ndarray:
    """Floating-point values spread over many binades (uint8 [n, e]): sign from
    bit 63, a binade 2^E with E uniform-ish in [lo_exp, hi_exp] from the bits
    above the mantissa, and a full random mantissa, so the value is
    +-(1 + m) * 2^E exactly (F32: 23 mantissa bits, F64: 52)."""
    span = np.uint64(hi_exp - lo_exp + 1)
    sign = np.where((z >> np.uint64(63)) != 0, -1.0, 1.0)
    if dtype == F32:
        m = (z & np.uint64(0x7FFFFF)).astype(np.float64) * 2.0 ** -23
        e = ((z >> np.uint64(23)) & np.uint64(0xFFFF)) % span
        v = (sign * (1.0 + m) * np.exp2(e.astype(np.float64) + lo_exp)).astype(np.float32)
    elif dtype == F64:
        m = (z & np.uint64((1 << 52) - 1)).astype(np.float64) * 2.0 ** -52
        e = ((z >> np.uint64(52)) & np.uint64(0x7FF)) % span
        v = sign * (1.0 + m) * np.exp2(e.astype(np.float64) + lo_exp)
    else:
        raise ValueError(dtype)
    return np.ascontiguousarray(v).view(np.uint8).reshape(len(z), v.dtype.itemsize)


def field_values(seed: int, stream: int, n: int, dtype: int, elem_bytes: int = 4,
                 start: int = 0) -> np.ndarray:
    return decode(splitmix64(seed, stream, start, n), dtype, elem_bytes)


def field_values_at(seed: int, stream: int, records, dtype: int, elem_bytes: int = 4) -> np.ndarray:
    """Values of the given records only (same draws as field_values)."""
    return decode(splitmix64_at(seed, stream, records), dtype, elem_bytes)


def uniform_index_at(seed: int, stream: int, counters, n: int) -> np.ndarray:
    """Draws number counters[k] of U[0, n), as uniform_index gives them."""
    z = splitmix64_at(seed, stream, counters)
    return (((z >> np.uint64(32)) * np.uint64(n)) >> np.uint64(32)).astype(np.int32)


def uniform_index(seed: int, stream: int, count: int, n: int, start: int = 0) -> np.ndarray:
    """count draws of U[0, n) as int32 (multiply-shift)."""
    z = splitmix64(seed, stream, start, count)
    return (((z >> np.uint64(32)) * np.uint64(n)) >> np.uint64(32)).astype(np.int32)


def record_matrix(seed: int, n: int, dtypes, elem_bytes, stream_base: int = 0,
                  start: int = 0) -> list:
    """Per-field raw bytes for records start..start+n-1 (field f uses stream base+f)."""
    return [field_values(seed, stream_base + f, n, dtypes[f], elem_bytes[f], start)
            for f in range(len(dtypes))]


def pack_aos(cols, n: int) -> np.ndarray:
    """Packed record image (fields in id order, no padding): uint8 [n, S]."""
    if not cols:
        return np.zeros((n, 0), np.uint8)
    return np.ascontiguousarray(np.concatenate(cols, axis=1))


# ---------------------------------------------------------------- torch side
def _t_srl(x, k: int):
    import torch
    return (x >> k) & torch.tensor((1 << (64 - k)) - 1, dtype=torch.int64, device=x.device)


def _signed(c: int) -> int:
    return c - (1 << 64) if c >= (1 << 63) else c


def splitmix64_torch(seed: int, stream: int, start: int, count: int, device):
    """Same draws as :func:`splitmix64`, computed with torch int64 (wrapping) ops."""
    import torch
    i = torch.arange(start + 1, start + count + 1, dtype=torch.int64, device=device)
    z = (i + _signed(_key(seed, stream))) * _signed(GAMMA)
    z = (z ^ _t_srl(z, 30)) * _signed(M1)
    z = (z ^ _t_srl(z, 27)) * _signed(M2)
    return z ^ _t_srl(z, 31)


def decode_torch(z, dtype: int, elem_bytes: int = 4):
    """torch form of :func:`decode`; returns uint8 [n, e] on z's device."""
    import torch
    if dtype == F32:
        v = (_t_srl(z, 40).to(torch.float64) * 2.0 ** -23 - 1.0).to(torch.float32)
    elif dtype == F64:
        v = _t_srl(z, 11).to(torch.float64) * 2.0 ** -52 - 1.0
    elif dtype == I32:
        v = _t_srl(z, 33).to(torch.int32)
    elif dtype == U32:
        v = _t_srl(z, 32).to(torch.int64).to(torch.int32)       # the low 32 bits of z >> 32
    elif dtype in (U16, I16):
        v = _t_srl(z, 48).to(torch.int16)
    elif dtype == U8:
        v = _t_srl(z, 56).to(torch.uint8)
    elif dtype == RAW:
        if elem_bytes == 8:
            v = z
        elif elem_bytes == 4:
            v = (z & 0xFFFFFFFF).to(torch.int32)
        elif elem_bytes == 2:
            v = (z & 0xFFFF).to(torch.int16)
        elif elem_bytes == 1:
            v = (z & 0xFF).to(torch.uint8)
        else:
            raise ValueError(elem_bytes)
    else:
        raise ValueError(dtype)
    return v.contiguous().view(torch.uint8).reshape(z.shape[0], -1)


def uniform_index_torch(seed: int, stream: int, count: int, n: int, device, start: int = 0):
    import torch
    z = splitmix64_torch(seed, stream, start, count, device)
    return ((_t_srl(z, 32) * n) >> 32).to(torch.int32)


# ---------------------------------------------------------------- workloads
class StructSpec:
    """A struct: per-field dtype code and element bytes, plus a record count."""

    def __init__(self, n: int, dtypes, elem_bytes):
        self.n = int(n)
        self.dtypes = list(dtypes)
        self.elem_bytes = list(elem_bytes)
        assert len(self.dtypes) == len(self.elem_bytes)

    @property
    def n_fields(self) -> int:
        return len(self.dtypes)

    @property
    def record_bytes(self) -> int:
        return sum(self.elem_bytes)


class SectionSpec:
    """A section: op code, read and write field ids, gather degree."""

    def __init__(self, op: int, read, write, degree: int = 0):
        self.op = op
        self.read = sorted(read)
        self.write = sorted(write)
        self.degree = degree

    def __repr__(self):
        return f"Section(op={self.op}, R={self.read}, W={self.write}, d={self.degree})"


# op codes (same numbering as the C-ABI's adha_op)
OP_GEN, OP_MULADD3, OP_SUB2, OP_SUM = 0, 1, 2, 3


def config1_struct(n: int = 65536) -> StructSpec:
    """Plain small workload: 8 fp32 fields."""
    return StructSpec(n, [F32] * 8, [4] * 8)


def config1_sections():
    return [SectionSpec(OP_MULADD3, [0, 1, 2], [3]),
            SectionSpec(OP_SUB2, [3, 4], [5]),
            SectionSpec(OP_SUM, list(range(7)), [7])]


def config2_struct(n: int = 1 << 26) -> StructSpec:
    """Single-remap workload: 8 fp32 then 8 int32 fields (64-byte records)."""
    return StructSpec(n, [F32] * 8 + [I32] * 8, [4] * 16)


def config2_aosoa():
    """AoSoA target: groups {0-3}, {4-7}, {8-15} with 64-record tiles."""
    gof = [0] * 4 + [1] * 4 + [2] * 8
    return gof, [64, 64, 64]


def config3_struct(n: int = 1 << 24) -> StructSpec:
    """Multi-section workload: 20 fp32, 8 int32, 4 fp64 (144-byte records)."""
    return StructSpec(n, [F32] * 20 + [I32] * 8 + [F64] * 4, [4] * 20 + [4] * 8 + [8] * 4)


def _shuffle(seed: int, stream: int, items):
    """Fisher-Yates shuffle driven by the generator."""
    items = list(items)
    z = splitmix64(seed, stream, 0, max(len(items), 1))
    for k in range(len(items) - 1, 0, -1):
        j = int(((int(z[k]) >> 32) * (k + 1)) >> 32)
        items[k], items[j] = items[j], items[k]
    return items


def random_program(seed: int, n_fields: int, k: int = 8, n_gather: int = 4, degree: int = 16,
                   r_range=(2, 10), w_range=(1, 2), stream0: int = 1000):
    """k GEN sections with random read sets (|R| ~ U{r_range}) and write sets drawn
    from the fields not read (|W| ~ U{w_range}); n_gather of them (chosen by a
    seeded shuffle) gather `degree` neighbours."""
    z = splitmix64(seed, stream0, 0, 4 * k)
    gathers = set(_shuffle(seed, stream0 + 1, range(k))[:n_gather])
    secs = []
    for s in range(k):
        nr = r_range[0] + int(((int(z[2 * s]) >> 32) * (r_range[1] - r_range[0] + 1)) >> 32)
        nw = w_range[0] + int(((int(z[2 * s + 1]) >> 32) * (w_range[1] - w_range[0] + 1)) >> 32)
        perm = _shuffle(seed, stream0 + 2 + s, range(n_fields))
        rd = perm[:nr]
        wr = perm[nr:nr + nw]
        secs.append(SectionSpec(OP_GEN, rd, wr, degree if s in gathers else 0))
    return secs


# op code of reductions (same numbering as the C-ABI's adha_op)
OP_REDUCE = 4
KMEANS_FEATURES, KMEANS_KEY, KMEANS_SCORE, KMEANS_K = 32, 32, 33, 5


def kmeans_struct(n: int = 8388608) -> StructSpec:
    """K-Means-shaped workload: 32 f32 features (ids 0-31), the cluster key
    (id 32, i32, drawn U[0, 5) from stream 77 by uniform_index) and one f32
    result field (id 33)."""
    return StructSpec(n, [F32] * 32 + [I32, F32], [4] * 34)


def kmeans_sections():
    """The two loops: a direct GEN over the features writing field 33, then a
    reduction of the features per cluster key (read, key, key count)."""
    return (SectionSpec(OP_GEN, list(range(KMEANS_FEATURES)), [KMEANS_SCORE]),
            (list(range(KMEANS_FEATURES)), KMEANS_KEY, KMEANS_K))


STENCIL7 = [(0, 0, 0), (-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0), (0, 0, -1), (0, 0, 1)]


def medical_struct(side: int = 256) -> StructSpec:
    """Medical-shaped workload: a side^3 image of 9 f32 fields (V1 V2 V3 U1
    U2 U3 S T interpT, ids 0-8)."""
    return StructSpec(side ** 3, [F32] * 9, [4] * 9)


def medical_narrow_struct(side: int = 256) -> StructSpec:
    """The Medical-shaped struct with narrow image fields: V1..V3 U16 (16-bit
    intensities), U1..U3 F32, S U8 (an 8-bit label), T I16 (a signed 16-bit
    value), interpT F32 -- 18 bytes per voxel, so fields of an interleaved
    group sit at offsets that are not multiples of 4."""
    n = side ** 3
    return StructSpec(n, [U16, U16, U16, F32, F32, F32, U8, I16, F32], [2, 2, 2, 4, 4, 4, 1, 2, 4])


def mixed_narrow_struct(n: int) -> StructSpec:
    """A struct of every typed element kind: U8, I16, F32, U16, F64, U32, I32,
    U8, F32, I16 (30 bytes per record)."""
    return StructSpec(n, [U8, I16, F32, U16, F64, U32, I32, U8, F32, I16], [1, 2, 4, 2, 8, 4, 4, 1, 4, 2])


def medical_sections():
    """Four loops: (read, write, stencil offsets or None for a direct loop).
    Two 7-point stencils (over U into V1, over V into U1) and two direct
    updates."""
    return [([3, 4, 5], [0], STENCIL7),
            ([0, 6, 7], [8], None),
            ([0, 1, 2], [3], STENCIL7),
            ([3, 4, 5, 8], [1, 2], None)]


def config4_arrays(seed: int = 4, n_arrays: int = 512, lo_log2: int = 10, hi_log2: int = 22):
    """Batched-remap workload: per array (n, elem_bytes[], target partition, tiles).

    n = floor(2^(lo + (hi-lo)*u)), F ~ U{4..24}, e in {4, 8}; target SoA with
    probability 1/2, otherwise consecutive field chunks of size g ~ U{2..8}
    with 64-record tiles."""
    out = []
    for a in range(n_arrays):
        z = splitmix64(seed, 2000 + a, 0, 64)
        u = (int(z[0]) >> 11) * 2.0 ** -53
        n = int(np.floor(2.0 ** (lo_log2 + (hi_log2 - lo_log2) * u)))
        nf = 4 + int(((int(z[1]) >> 32) * 21) >> 32)
        eb = [4 if (int(z[2 + f]) >> 63) == 0 else 8 for f in range(nf)]
        soa = (int(z[30]) >> 63) == 0
        if soa:
            gof = list(range(nf))
            tiles = [1] * nf
        else:
            g = 2 + int(((int(z[31]) >> 32) * 7) >> 32)
            gof = [f // g for f in range(nf)]
            tiles = [64] * (max(gof) + 1)
        out.append(dict(n=n, elem_bytes=eb, target_gof=gof, target_tiles=tiles))
    return out
