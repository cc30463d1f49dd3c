"""CPU oracle for the data-layout hot path.  TEST INFRASTRUCTURE ONLY.

Only the tests, the package's smoke check and the benchmark's CPU-baseline
leg may import this package.  It shares no code with the library: the
address map (layout.py), remap and section loops (adha_oracle.c), the
two-level selection (planner.py) and the cost-model network (mlp.py) are
written out from their definitions, slowly and plainly.

Parity status per function (what pins each one is listed in its tests):
  layout.Layout          pinned (closed forms, bijectivity, Table 2 encodings)
  remap                  pinned (numpy transpose, round trip, composition)
  section                pinned (numpy float32 ops, sequential sums, invariants)
  planner.affinity       pinned (hand-derived weights)
  planner.ods_greedy     pinned (Table 3 split, brute-force partitions)
  planner.pdl_dp         pinned (brute-force enumeration, networkx)
  mlp                    pinned (finite differences, least squares)
  stencil_index          pinned (hand-listed neighbours of a small grid)
  reduce.reduce          pinned (exact rounding by hand, closed form, brute force)
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

from .layout import Layout, aos, soa, from_partition  # noqa: F401

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "adha_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

F32, F64, I32, RAW, U32, U8, U16, I16 = 0, 1, 2, 3, 4, 5, 6, 7
OP_GEN, OP_MULADD3, OP_SUB2, OP_SUM = 0, 1, 2, 3


def build(force: bool = False) -> str:
    """Compile the C oracle with gcc (-O2 -ffp-contract=off, no fast-math)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math",
                               "-fPIC", "-shared", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        L.orc_remap.argtypes = [ctypes.c_int32, P, P, P, P, ctypes.c_int64, ctypes.c_int64]
        L.orc_remap.restype = None
        L.orc_section.argtypes = [ctypes.c_int32, ctypes.c_int64, P, P, ctypes.c_int32, P,
                                  ctypes.c_int32, P, ctypes.c_int32, P, P,
                                  ctypes.c_int64, ctypes.c_int64]
        L.orc_section.restype = ctypes.c_int64
        L.orc_layout_addr.argtypes = [P, ctypes.c_int32, ctypes.c_int64]
        L.orc_layout_addr.restype = ctypes.c_uint64
        _lib = L
    return _lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def remap(src_layout: Layout, src: np.ndarray, dst_layout: Layout,
          r_begin: int = 0, r_end=None, out: np.ndarray = None) -> np.ndarray:
    """Remap a whole buffer (zero-filled destination, then every (r, f) copied)."""
    n = src_layout.n
    r_end = n if r_end is None else r_end
    src = np.ascontiguousarray(src, dtype=np.uint8)
    if out is None:
        out = np.zeros(dst_layout.nbytes, np.uint8)
    sd = np.ascontiguousarray(src_layout.desc())
    dd = np.ascontiguousarray(dst_layout.desc())
    lib().orc_remap(len(src_layout.elem_bytes), _p(sd), _p(src), _p(dd), _p(out), r_begin, r_end)
    return out


def remap_in_place(src_layout: Layout, dst_layout: Layout, buf: np.ndarray) -> np.ndarray:
    """A remap inside one buffer that moves only what changes.

    Both layouts describe where the struct's groups sit in `buf` (placed
    layouts).  A group of dst_layout that src_layout holds with the same
    fields, tile and base stays as it is.  Every other group of dst_layout is
    written: its region is zeroed, then each of its (record, field) elements
    is copied from where src_layout holds it.  All other bytes of the buffer
    keep their value.  Returns the new buffer (the input is not changed)."""
    out = np.array(buf, dtype=np.uint8, copy=True)
    stay = set()
    for g, grp in enumerate(dst_layout.groups):
        for h, other in enumerate(src_layout.groups):
            if other == grp and src_layout.base[h] == dst_layout.base[g]:
                stay.add(g)
    moving = [f for f in range(len(dst_layout.elem_bytes)) if dst_layout.group_of[f] not in stay]
    for g in range(len(dst_layout.groups)):
        if g not in stay:
            a, b = dst_layout.region(g)
            out[a:b] = 0
    if moving and src_layout.n:
        sd = np.ascontiguousarray(src_layout.desc()[moving])
        dd = np.ascontiguousarray(dst_layout.desc()[moving])
        src = np.ascontiguousarray(buf, dtype=np.uint8)
        lib().orc_remap(len(moving), _p(sd), _p(src), _p(dd), _p(out), 0, src_layout.n)
    return out


def section(layout: Layout, dtypes, op: int, read, write, degree: int, idx, buf: np.ndarray,
            r_begin: int = 0, r_end=None) -> int:
    """Run one section in place on `buf` (records [r_begin, r_end)); returns the
    number of out-of-range gather indices seen."""
    n = layout.n
    r_end = n if r_end is None else r_end
    d = np.ascontiguousarray(layout.desc())
    dt = np.ascontiguousarray(np.asarray(dtypes, np.int32))
    rd = np.ascontiguousarray(np.asarray(sorted(read), np.int32))
    wr = np.ascontiguousarray(np.asarray(sorted(write), np.int32))
    ix = np.ascontiguousarray(np.asarray(idx if idx is not None else np.zeros(1, np.int32),
                                         np.int32))
    bad = lib().orc_section(op, n, _p(d), _p(dt), len(rd), _p(rd), len(wr), _p(wr), degree,
                            _p(ix), _p(buf), r_begin, r_end)
    if bad < 0:
        raise ValueError("too many terms per record")
    return int(bad)


def stencil_index(nx: int, ny: int, nz: int, offsets) -> np.ndarray:
    """The index array a stencil stands for (section 3: the Medical loops run
    over a 3-D image): record r = x + nx*(y + ny*z), neighbour j at
    (x+dx, y+dy, z+dz), written as -1 (left out) when outside the grid.
    Feed it to section() and ignore the count of left-out neighbours."""
    n = nx * ny * nz
    r = np.arange(n, dtype=np.int64)
    x, y, z = r % nx, (r // nx) % ny, r // (nx * ny)
    out = np.empty((n, len(offsets)), np.int32)
    for j, (dx, dy, dz) in enumerate(offsets):
        xx, yy, zz = x + dx, y + dy, z + dz
        inside = (xx >= 0) & (xx < nx) & (yy >= 0) & (yy < ny) & (zz >= 0) & (zz < nz)
        out[:, j] = np.where(inside, xx + nx * (yy + ny * zz), -1)
    return out.reshape(-1)


def pack(layout: Layout, cols) -> np.ndarray:
    """Buffer in `layout` holding per-field element bytes cols[f] (uint8 [N, e_f])."""
    buf = np.zeros(layout.nbytes, np.uint8)
    r = np.arange(layout.n, dtype=np.int64)
    for f, e in enumerate(layout.elem_bytes):
        a = layout.addr_vec(r, f)
        for b in range(e):
            buf[a + b] = cols[f][:, b]
    return buf


def unpack(layout: Layout, buf: np.ndarray, f: int, records=None) -> np.ndarray:
    """Element bytes of field f (uint8 [len(records), e_f])."""
    r = np.arange(layout.n, dtype=np.int64) if records is None else np.asarray(records, np.int64)
    e = layout.elem_bytes[f]
    a = layout.addr_vec(r, f)
    return np.stack([buf[a + b] for b in range(e)], axis=1) if len(r) else np.zeros((0, e), np.uint8)


def padding_mask(layout: Layout) -> np.ndarray:
    """True at every byte of the layout that no (record, field) owns."""
    m = np.ones(layout.nbytes, bool)
    r = np.arange(layout.n, dtype=np.int64)
    for f, e in enumerate(layout.elem_bytes):
        a = layout.addr_vec(r, f)
        for b in range(e):
            m[a + b] = False
    return m
