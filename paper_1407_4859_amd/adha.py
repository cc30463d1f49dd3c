"""Thin Python binding of libadha's C-ABI (argument marshalling only).

Every call goes straight to the library; every step of the hot path runs in
its HIP kernels.  torch provides device memory (tensors whose data_ptr() is
passed as a plain device pointer) and streams (passed as hipStream_t).  The
library must be built (``python -m paper_1407_4859_amd.build``); there is
no fallback when it is missing.
"""
from __future__ import annotations

import ctypes
import os
import re

import torch  # loads the HIP runtime that libadha then shares

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libadha.so")
# the learned cost model trained on an MI355X's own timings (train_costmodel.py)
DEFAULT_MODEL = os.path.join(HERE, "models", "costmodel_mi355x.adha")
HEADER = os.path.join(os.path.dirname(HERE), "include", "adha.h")

OK, WARN_FALLBACK = 0, 1
ERR_INVALID, ERR_OOM, ERR_DEVICE, ERR_STATE, ERR_UNSUPPORTED, ERR_IO = -1, -2, -3, -4, -5, -6
F32, F64, I32, RAW, U32, U8, U16, I16 = 0, 1, 2, 3, 4, 5, 6, 7
OP_GEN, OP_MULADD3, OP_SUB2, OP_SUM, OP_REDUCE = 0, 1, 2, 3, 4
MAX_REDUCE_CELLS = 4096
COST_MEASURED, COST_ANALYTIC, COST_LEARNED = 0, 1, 2
CAT_AOS_SOA, CAT_FULL = 0, 1
INIT_FREE, INIT_AOS, INIT_HOST_AOS = 0, 1, 2
BATCH_GRAPH, BATCH_SEPARATE = 1, 2
OPT_SPAN_GATHER, OPT_REDUCE_WG_PER_CU, OPT_REDUCE_COMPENSATED, OPT_HOST_THREADS = 1, 2, 3, 4
DEVICES_GPU, DEVICES_GPU_HOST = 0, 1
N_FEATURES = 16
MLP_PARAMS = 64 * 16 + 64 + 64 * 64 + 64 + 64 * 64 + 64 + 64 + 1


class AdhaError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"[{status}] {msg}")
        self.status = status


class TileShape(ctypes.Structure):
    _fields_ = [("tile_records", ctypes.c_uint32), ("slots", ctypes.c_uint32),
                ("pad_shift", ctypes.c_uint32), ("wg_per_cu", ctypes.c_uint32),
                ("order", ctypes.c_uint32), ("nontemporal", ctypes.c_uint32)]


class RemapItem(ctypes.Structure):
    _fields_ = [("src_layout", ctypes.c_void_p), ("src", ctypes.c_void_p), ("src_cap", ctypes.c_uint64),
                ("dst_layout", ctypes.c_void_p), ("dst", ctypes.c_void_p), ("dst_cap", ctypes.c_uint64)]


class RemapInfo(ctypes.Structure):
    _fields_ = [("shape", TileShape), ("full_tiles", ctypes.c_uint64), ("tail_bytes", ctypes.c_uint64),
                ("descriptor_bytes", ctypes.c_uint64), ("grid", ctypes.c_uint64), ("lds_bytes", ctypes.c_uint32),
                ("byte_path", ctypes.c_uint32)]


class PlanOpts(ctypes.Structure):
    _fields_ = [("cost", ctypes.c_int), ("catalogue", ctypes.c_int), ("cap_bytes", ctypes.c_uint32),
                ("init", ctypes.c_int), ("reps", ctypes.c_uint32), ("devices", ctypes.c_int),
                ("pair_remaps", ctypes.c_uint32), ("verify_rounds", ctypes.c_uint32)]


class TrainOpts(ctypes.Structure):
    _fields_ = [("n_samples", ctypes.c_uint32), ("epochs", ctypes.c_uint32), ("batch", ctypes.c_uint32),
                ("lr", ctypes.c_float), ("seed", ctypes.c_uint64), ("min_log2_n", ctypes.c_int32),
                ("max_log2_n", ctypes.c_int32), ("reps", ctypes.c_uint32), ("progress_every", ctypes.c_uint32),
                ("ensemble", ctypes.c_uint32)]


class TrainReport(ctypes.Structure):
    _fields_ = [("gen_seconds", ctypes.c_double), ("train_seconds", ctypes.c_double),
                ("train_loss", ctypes.c_double), ("val_loss", ctypes.c_double),
                ("val_mape", ctypes.c_double), ("n_train", ctypes.c_uint32), ("n_val", ctypes.c_uint32)]


P = ctypes.c_void_p
PP = ctypes.POINTER(ctypes.c_void_p)
U32, I32T, U64, I64, DBL, FLT = (ctypes.c_uint32, ctypes.c_int32, ctypes.c_uint64, ctypes.c_int64,
                                  ctypes.c_double, ctypes.c_float)
_SIGS = {
    "adha_status_string": ([I32T], ctypes.c_char_p),
    "adha_last_error": ([], ctypes.c_char_p),
    "adha_version": ([], I32T),
    "adha_ctx_create": ([I32T, PP], I32T),
    "adha_ctx_destroy": ([P], I32T),
    "adha_ctx_check": ([P, P], I32T),
    "adha_ctx_cu_count": ([P, ctypes.POINTER(I32T)], I32T),
    "adha_ctx_set_option": ([P, ctypes.c_int, I64], I32T),
    "adha_struct_create": ([I64, PP], I32T),
    "adha_struct_add_field": ([P, ctypes.c_int, U32, ctypes.POINTER(I32T)], I32T),
    "adha_struct_destroy": ([P], I32T),
    "adha_struct_info": ([P, ctypes.POINTER(I64), ctypes.POINTER(I32T), ctypes.POINTER(U32)], I32T),
    "adha_layout_create": ([P, U32, P, P, PP], I32T),
    "adha_layout_aos": ([P, PP], I32T),
    "adha_layout_soa": ([P, PP], I32T),
    "adha_layout_destroy": ([P], I32T),
    "adha_layout_nbytes": ([P, ctypes.POINTER(U64)], I32T),
    "adha_layout_addr": ([P, I64, I32T, ctypes.POINTER(U64)], I32T),
    "adha_layout_groups": ([P, ctypes.POINTER(U32), P, P], I32T),
    "adha_layout_equal": ([P, P, ctypes.POINTER(I32T)], I32T),
    "adha_remap": ([P, P, P, U64, P, P, U64, P], I32T),
    "adha_remap_batched": ([P, U32, P, U32, P], I32T),
    "adha_remap_set_shape": ([P, P, P, ctypes.POINTER(TileShape)], I32T),
    "adha_remap_get_shape": ([P, P, P, ctypes.POINTER(TileShape)], I32T),
    "adha_remap_describe": ([P, P, I32T, ctypes.POINTER(RemapInfo)], I32T),
    "adha_tune_remap": ([P, P, P, U64, P, P, U64, U32, P, ctypes.POINTER(TileShape), ctypes.POINTER(DBL),
                         ctypes.POINTER(DBL)], I32T),
    "adha_tune_batched": ([P, U32, P, U32, P, ctypes.POINTER(U32), ctypes.POINTER(TileShape),
                           ctypes.POINTER(DBL), ctypes.POINTER(DBL)], I32T),
    "adha_tune_save": ([P, ctypes.c_char_p], I32T),
    "adha_tune_load": ([P, ctypes.c_char_p], I32T),
    "adha_section_create": ([P, ctypes.c_int, U32, P, U32, P, U32, PP], I32T),
    "adha_section_create_reduce": ([P, U32, P, ctypes.c_int32, U32, P, U64, PP], I32T),
    "adha_section_create_stencil": ([P, U32, P, U32, P, U32, U32, U32, U32, P, PP], I32T),
    "adha_section_destroy": ([P], I32T),
    "adha_section_run": ([P, P, P, P, U64, P, U64, P], I32T),
    "adha_section_run_static": ([P, P, P, P, U64, P, U64, P], I32T),
    "adha_layout_place": ([P, U32, P, PP], I32T),
    "adha_layout_bases": ([P, P], I32T),
    "adha_remap_in_place": ([P, P, P, P, U64, P], I32T),
    "adha_plan_arena": ([P, ctypes.POINTER(U64), PP, PP], I32T),
    "adha_run_placed": ([P, P, P, U64, P, U64, P], I32T),
    "adha_plan_placed": ([P, U32, PP], I32T),
    "adha_plan_with_init": ([P, ctypes.c_int, PP], I32T),
    "adha_plan_verified": ([P, ctypes.POINTER(U32)], I32T),
    "adha_probe_stream": ([P, U32, P, P, U64, U32, P, ctypes.POINTER(DBL)], I32T),
    "adha_probe_gather": ([P, P, U64, U64, U32, P, U64, P, U32, P, ctypes.POINTER(DBL)], I32T),
    "adha_section_bytes": ([P, ctypes.POINTER(U64)], I32T),
    "adha_section_effective_bytes": ([P, P, ctypes.POINTER(ctypes.c_double)], I32T),
    "adha_host_section_run": ([P, P, P, U64, P, U64, P, U64, U32, ctypes.POINTER(U64)], I32T),
    "adha_host_remap": ([P, P, U64, P, P, U64, U32], I32T),
    "adha_program_create": ([P, U32, P, PP], I32T),
    "adha_program_destroy": ([P], I32T),
    "adha_affinity": ([P, U32, U32, P], I32T),
    "adha_ods": ([P, U32, U32, U32, U32, PP], I32T),
    "adha_pdl_solve": ([U32, U32, P, P, P, P, ctypes.POINTER(DBL)], I32T),
    "adha_plan_opts_default": ([ctypes.POINTER(PlanOpts)], I32T),
    "adha_plan_create": ([P, P, ctypes.POINTER(PlanOpts), P, U64, P, PP], I32T),
    "adha_plan_uniform": ([P, P, PP], I32T),
    "adha_plan_destroy": ([P], I32T),
    "adha_plan_n_candidates": ([P, ctypes.POINTER(U32)], I32T),
    "adha_plan_candidate": ([P, U32, PP], I32T),
    "adha_plan_choice": ([P, U32, ctypes.POINTER(U32)], I32T),
    "adha_plan_cost": ([P, ctypes.POINTER(DBL)], I32T),
    "adha_plan_tables": ([P, P, P], I32T),
    "adha_plan_time": ([P, ctypes.POINTER(DBL)], I32T),
    "adha_run": ([P, P, P, P, P, U64, P, U64, P, PP, ctypes.POINTER(I32T)], I32T),
    "adha_run_hetero": ([P, P, P, I32T, P, P, P, P, U64, P, P, U64, P, PP, ctypes.POINTER(I32T),
                         ctypes.POINTER(I32T)], I32T),
    "adha_plan_explicit": ([P, P, P, PP], I32T),
    "adha_program_set_flow": ([P, U32, P, P], I32T),
    "adha_flow_solve": ([U32, U32, P, P, P, U32, P, P, P, P, P, ctypes.POINTER(ctypes.c_double)], I32T),
    "adha_plan_join": ([P, U32, ctypes.POINTER(U32)], I32T),
    "adha_run_flow": ([P, P, P, P, P, U64, P, U64, P, U32, P, PP, ctypes.POINTER(I32T)], I32T),
    "adha_plan_device": ([P, U32, ctypes.POINTER(I32T)], I32T),
    "adha_plan_nodes": ([P, ctypes.POINTER(U32)], I32T),
    "adha_plan_node_tables": ([P, P, P], I32T),
    "adha_features": ([P, P, P], I32T),
    "adha_mlp_forward": ([P, P, P, U32, P, P], I32T),
    "adha_mlp_backward": ([P, P, P, P, U32, P, P, P], I32T),
    "adha_mlp_adam": ([P, P, P, P, P, FLT, FLT, FLT, FLT, U32, P], I32T),
    "adha_train_opts_default": ([ctypes.POINTER(TrainOpts)], I32T),
    "adha_costmodel_train": ([P, ctypes.POINTER(TrainOpts), ctypes.POINTER(TrainReport)], I32T),
    "adha_costmodel_save": ([P, ctypes.c_char_p], I32T),
    "adha_costmodel_load": ([P, ctypes.c_char_p], I32T),
    "adha_costmodel_predict": ([P, P, P, ctypes.POINTER(DBL)], I32T),
}

_lib = None


def header_symbols():
    """Function names the C header declares."""
    with open(HEADER) as fh:
        txt = fh.read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(adha_[a-z0-9_]+)\s*\(", txt)))


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with python -m paper_1407_4859_amd.build")
        L = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in _SIGS.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def check(st: int) -> int:
    if st < 0:
        msg = lib().adha_last_error().decode()
        raise AdhaError(st, msg)
    return st


def _u32(vals):
    arr = (ctypes.c_uint32 * max(1, len(vals)))(*vals)
    return arr


def _i32(vals):
    return (ctypes.c_int32 * max(1, len(vals)))(*vals)


def stream_ptr(stream=None):
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


def _dev(t):
    """(pointer, capacity in bytes) of a device tensor (or (None, 0))."""
    if t is None:
        return None, 0
    return ctypes.c_void_p(t.data_ptr()), t.numel() * t.element_size()


class Ctx:
    def __init__(self, device: int = 0):
        h = ctypes.c_void_p()
        check(lib().adha_ctx_create(device, ctypes.byref(h)))
        self.h = h

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.adha_ctx_destroy(self.h)
            self.h = None

    def check(self, stream=None):
        return check(lib().adha_ctx_check(self.h, stream_ptr(stream)))

    def set_option(self, opt: int, value: int):
        check(lib().adha_ctx_set_option(self.h, opt, value))

    @property
    def cu_count(self):
        v = ctypes.c_int32()
        check(lib().adha_ctx_cu_count(self.h, ctypes.byref(v)))
        return v.value


class Struct:
    def __init__(self, n: int, dtypes, elem_bytes=None):
        h = ctypes.c_void_p()
        check(lib().adha_struct_create(n, ctypes.byref(h)))
        self.h = h
        self.n = n
        self.dtypes = list(dtypes)
        self.elem_bytes = list(elem_bytes) if elem_bytes is not None else \
            [{F64: 8, U16: 2, I16: 2, U8: 1}.get(d, 4) for d in dtypes]
        for d, e in zip(self.dtypes, self.elem_bytes):
            fid = ctypes.c_int32()
            check(lib().adha_struct_add_field(h, d, e, ctypes.byref(fid)))

    @classmethod
    def from_spec(cls, spec):
        return cls(spec.n, spec.dtypes, spec.elem_bytes)

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.adha_struct_destroy(self.h)
            self.h = None


class Layout:
    def __init__(self, h, owned=True, keep=None):
        self.h = h
        self.owned = owned
        self.keep = keep  # an owner that must outlive a borrowed handle

    @classmethod
    def create(cls, st: Struct, group_of_field, tile_of_group):
        h = ctypes.c_void_p()
        check(lib().adha_layout_create(st.h, len(tile_of_group), _u32(group_of_field),
                                       _u32(tile_of_group), ctypes.byref(h)))
        return cls(h)

    @classmethod
    def aos(cls, st: Struct):
        h = ctypes.c_void_p()
        check(lib().adha_layout_aos(st.h, ctypes.byref(h)))
        return cls(h)

    @classmethod
    def soa(cls, st: Struct):
        h = ctypes.c_void_p()
        check(lib().adha_layout_soa(st.h, ctypes.byref(h)))
        return cls(h)

    def __del__(self):
        if getattr(self, "owned", False) and getattr(self, "h", None) and _lib is not None:
            _lib.adha_layout_destroy(self.h)
            self.h = None

    @property
    def nbytes(self) -> int:
        v = ctypes.c_uint64()
        check(lib().adha_layout_nbytes(self.h, ctypes.byref(v)))
        return v.value

    def addr(self, r: int, f: int) -> int:
        v = ctypes.c_uint64()
        check(lib().adha_layout_addr(self.h, r, f, ctypes.byref(v)))
        return v.value

    def groups(self, n_fields: int):
        ng = ctypes.c_uint32()
        gof = (ctypes.c_uint32 * n_fields)()
        tog = (ctypes.c_uint32 * n_fields)()
        check(lib().adha_layout_groups(self.h, ctypes.byref(ng), gof, tog))
        return list(gof), list(tog)[: ng.value]

    def equals(self, other) -> bool:
        v = ctypes.c_int32()
        check(lib().adha_layout_equal(self.h, other.h, ctypes.byref(v)))
        return bool(v.value)

    def n_groups(self) -> int:
        ng = ctypes.c_uint32()
        check(lib().adha_layout_groups(self.h, ctypes.byref(ng), None, None))
        return ng.value

    def place(self, bases):
        """A placed copy (adha_layout_place): one base per group."""
        h = ctypes.c_void_p()
        arr = (ctypes.c_uint64 * max(1, len(bases)))(*[int(b) for b in bases])
        check(lib().adha_layout_place(self.h, len(bases), arr, ctypes.byref(h)))
        return Layout(h)

    def bases(self):
        ng = self.n_groups()
        arr = (ctypes.c_uint64 * max(1, ng))()
        check(lib().adha_layout_bases(self.h, arr))
        return list(arr)[:ng]


class Section:
    def __init__(self, st: Struct, op: int, read, write, degree: int = 0):
        h = ctypes.c_void_p()
        check(lib().adha_section_create(st.h, op, len(read), _i32(read), len(write), _i32(write),
                                        degree, ctypes.byref(h)))
        self.h = h
        self.op, self.read, self.write, self.degree = op, sorted(read), sorted(write), degree

    @classmethod
    def from_spec(cls, st: Struct, spec):
        if spec.op == OP_REDUCE:
            raise ValueError("reduction specs need a result table: use Section.reduce")
        return cls(st, spec.op, spec.read, spec.write, spec.degree)

    @classmethod
    def stencil(cls, st: Struct, read, write, grid, offsets):
        """A GEN gather over grid neighbours: grid = (nx, ny, nz), offsets a
        list of (dx, dy, dz)."""
        flat = [int(v) for o in offsets for v in o]
        h = ctypes.c_void_p()
        check(lib().adha_section_create_stencil(st.h, len(read), _i32(read), len(write), _i32(write),
                                                grid[0], grid[1], grid[2], len(offsets), _i32(flat),
                                                ctypes.byref(h)))
        self = cls.__new__(cls)
        self.h = h
        self.op, self.read, self.write, self.degree = OP_GEN, sorted(read), sorted(write), len(offsets)
        self.grid, self.offsets = tuple(grid), [tuple(o) for o in offsets]
        return self

    @classmethod
    def reduce(cls, st: Struct, read, key: int, n_keys: int, out):
        """A reduction of the read fields over the records, per key (key -1:
        one row); `out` is a device tensor of at least n_keys*(len(read)+1)
        eight-byte cells that every run overwrites."""
        op, oc = _dev(out)
        h = ctypes.c_void_p()
        check(lib().adha_section_create_reduce(st.h, len(read), _i32(read), key, n_keys, op, oc,
                                               ctypes.byref(h)))
        self = cls.__new__(cls)
        self.h = h
        self.op, self.read, self.write, self.degree = OP_REDUCE, sorted(read), [], 0
        self.key, self.n_keys, self.out = key, n_keys, out
        return self

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.adha_section_destroy(self.h)
            self.h = None

    @property
    def bytes(self) -> int:
        v = ctypes.c_uint64()
        check(lib().adha_section_bytes(self.h, ctypes.byref(v)))
        return v.value

    def effective_bytes(self, layout: Layout) -> float:
        v = ctypes.c_double()
        check(lib().adha_section_effective_bytes(self.h, layout.h, ctypes.byref(v)))
        return v.value

    def features(self, layout: Layout):
        out = (ctypes.c_float * N_FEATURES)()
        check(lib().adha_features(self.h, layout.h, out))
        return list(out)


class Program:
    def __init__(self, st: Struct, sections):
        h = ctypes.c_void_p()
        arr = (ctypes.c_void_p * len(sections))(*[s.h.value for s in sections])
        check(lib().adha_program_create(st.h, len(sections), arr, ctypes.byref(h)))
        self.h = h
        self.sections = list(sections)
        self.n_fields = len(st.dtypes)

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.adha_program_destroy(self.h)
            self.h = None

    def affinity(self, first: int, last: int):
        F = self.n_fields
        w = (ctypes.c_uint64 * (F * F))()
        check(lib().adha_affinity(self.h, first, last, w))
        return [[w[a * F + b] for b in range(F)] for a in range(F)]

    def set_flow(self, tokens, probs=()):
        """Branches: tokens are section indices and TOK_IF / TOK_ELSE /
        TOK_END; probs holds one probability per TOK_IF."""
        self.flow = (list(tokens), list(probs))
        pr = (ctypes.c_double * len(probs))(*probs) if probs else None
        check(lib().adha_program_set_flow(self.h, len(tokens), _i32(tokens) if tokens else None, pr))

    def ods(self, first: int, last: int, cap_bytes: int, tile: int = 1) -> Layout:
        h = ctypes.c_void_p()
        check(lib().adha_ods(self.h, first, last, cap_bytes, tile, ctypes.byref(h)))
        return Layout(h)


TOK_IF, TOK_ELSE, TOK_END = -1, -2, -3


def flow_solve(T, R, tokens, probs=(), R0=None):
    """(cost, start node, node per section, join node per branch)."""
    k, C = len(T), len(T[0])
    Tf = (ctypes.c_double * (k * C))(*[v for row in T for v in row])
    Rf = (ctypes.c_double * (C * C))(*[v for row in R for v in row])
    R0f = (ctypes.c_double * C)(*R0) if R0 is not None else None
    nb = sum(1 for t in tokens if t == TOK_IF)
    node = (ctypes.c_uint32 * k)()
    join = (ctypes.c_uint32 * max(1, nb))()
    start = ctypes.c_uint32()
    cost = ctypes.c_double()
    pr = (ctypes.c_double * len(probs))(*probs) if probs else None
    check(lib().adha_flow_solve(k, C, Tf, Rf, R0f, len(tokens), _i32(tokens), pr, node, join,
                                ctypes.byref(start), ctypes.byref(cost)))
    return cost.value, start.value, list(node), list(join)[:nb]


def pdl_solve(T, R, R0=None):
    k, C = len(T), len(T[0])
    Ta = (ctypes.c_double * (k * C))(*[v for row in T for v in row])
    Ra = (ctypes.c_double * (C * C))(*[v for row in R for v in row])
    R0a = (ctypes.c_double * C)(*R0) if R0 is not None else None
    path = (ctypes.c_uint32 * k)()
    cost = ctypes.c_double()
    check(lib().adha_pdl_solve(k, C, Ta, Ra, R0a, path, ctypes.byref(cost)))
    return cost.value, list(path)


def plan_opts(**kw) -> PlanOpts:
    o = PlanOpts()
    check(lib().adha_plan_opts_default(ctypes.byref(o)))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


class Plan:
    def __init__(self, h, k: int, status: int = OK):
        self.h = h
        self.k = k
        self.status = status

    @classmethod
    def create(cls, ctx: Ctx, prog: Program, opts: PlanOpts = None, idx=None, stream=None):
        opts = opts or plan_opts()
        h = ctypes.c_void_p()
        ip, icap = _dev(idx)
        st = check(lib().adha_plan_create(ctx.h, prog.h, ctypes.byref(opts), ip, icap // 4,
                                          stream_ptr(stream), ctypes.byref(h)))
        return cls(h, len(prog.sections), st)

    @property
    def verified(self) -> int:
        v = ctypes.c_uint32()
        check(lib().adha_plan_verified(self.h, ctypes.byref(v)))
        return v.value

    def with_init(self, init: int):
        """adha_plan_with_init: the same tables solved for another start."""
        h = ctypes.c_void_p()
        check(lib().adha_plan_with_init(self.h, init, ctypes.byref(h)))
        return Plan(h, self.k)

    @classmethod
    def uniform(cls, prog: Program, layout: Layout):
        h = ctypes.c_void_p()
        check(lib().adha_plan_uniform(prog.h, layout.h, ctypes.byref(h)))
        return cls(h, len(prog.sections))

    @classmethod
    def explicit(cls, prog: Program, layouts, devices=None):
        """A plan given section by section (devices: 0 the GPU, 1 the host)."""
        h = ctypes.c_void_p()
        arr = (ctypes.c_void_p * len(layouts))(*[l.h.value for l in layouts])
        dv = _i32(devices) if devices is not None else None
        check(lib().adha_plan_explicit(prog.h, arr, dv, ctypes.byref(h)))
        return cls(h, len(prog.sections))

    def joins(self, n_branches: int):
        out = []
        for b in range(n_branches):
            v = ctypes.c_uint32()
            check(lib().adha_plan_join(self.h, b, ctypes.byref(v)))
            out.append(v.value)
        return out

    def devices(self):
        out = []
        for s in range(self.k):
            v = ctypes.c_int32()
            check(lib().adha_plan_device(self.h, s, ctypes.byref(v)))
            out.append(v.value)
        return out

    def node_tables(self):
        M = ctypes.c_uint32()
        check(lib().adha_plan_nodes(self.h, ctypes.byref(M)))
        m = M.value
        T = (ctypes.c_double * (self.k * m))()
        R = (ctypes.c_double * (m * m))()
        check(lib().adha_plan_node_tables(self.h, T, R))
        return ([[T[s * m + c] for c in range(m)] for s in range(self.k)],
                [[R[a * m + b] for b in range(m)] for a in range(m)])

    def __del__(self):
        if getattr(self, "h", None) and _lib is not None:
            _lib.adha_plan_destroy(self.h)
            self.h = None

    @property
    def n_candidates(self) -> int:
        v = ctypes.c_uint32()
        check(lib().adha_plan_n_candidates(self.h, ctypes.byref(v)))
        return v.value

    def candidate(self, c: int) -> Layout:
        h = ctypes.c_void_p()
        check(lib().adha_plan_candidate(self.h, c, ctypes.byref(h)))
        return Layout(h, owned=False, keep=self)

    def choices(self):
        out = []
        for s in range(self.k):
            v = ctypes.c_uint32()
            check(lib().adha_plan_choice(self.h, s, ctypes.byref(v)))
            out.append(v.value)
        return out

    @property
    def cost(self) -> float:
        v = ctypes.c_double()
        check(lib().adha_plan_cost(self.h, ctypes.byref(v)))
        return v.value

    @property
    def seconds(self) -> float:
        v = ctypes.c_double()
        check(lib().adha_plan_time(self.h, ctypes.byref(v)))
        return v.value

    def tables(self):
        C = self.n_candidates
        T = (ctypes.c_double * (self.k * C))()
        R = (ctypes.c_double * (C * C))()
        check(lib().adha_plan_tables(self.h, T, R))
        return ([[T[s * C + c] for c in range(C)] for s in range(self.k)],
                [[R[a * C + b] for b in range(C)] for a in range(C)])


def remap(ctx: Ctx, src_l: Layout, src, dst_l: Layout, dst, stream=None):
    sp, sc = _dev(src)
    dp, dc = _dev(dst)
    check(lib().adha_remap(ctx.h, src_l.h, sp, sc, dst_l.h, dp, dc, stream_ptr(stream)))


class BatchItems:
    """The C item array of a batch, marshalled once, for callers that replay
    one batch many times (its tensors and layouts must stay alive)."""

    def __init__(self, items):
        self.n = len(items)
        self.arr = _items(items)


def remap_batched(ctx: Ctx, items, flags: int = 0, stream=None):
    """items: (src layout, src tensor, dst layout, dst tensor) tuples, or a
    BatchItems."""
    b = items if isinstance(items, BatchItems) else BatchItems(items)
    check(lib().adha_remap_batched(ctx.h, b.n, b.arr, flags, stream_ptr(stream)))


def set_shape(ctx: Ctx, src_l: Layout, dst_l: Layout, tile_records=0, slots=0, pad_shift=0, wg_per_cu=0,
              order=0, nontemporal=0):
    """Force a tile shape (0 = automatic; order 1 contiguous / 2 strided;
    nontemporal 1 off / 2 on)."""
    s = TileShape(tile_records, slots, pad_shift, wg_per_cu, order, nontemporal)
    check(lib().adha_remap_set_shape(ctx.h, src_l.h, dst_l.h, ctypes.byref(s)))


def get_shape(ctx: Ctx, src_l: Layout, dst_l: Layout) -> dict:
    s = TileShape()
    check(lib().adha_remap_get_shape(ctx.h, src_l.h, dst_l.h, ctypes.byref(s)))
    return dict(tile_records=s.tile_records, slots=s.slots, pad_shift=s.pad_shift, wg_per_cu=s.wg_per_cu,
                order=s.order, nontemporal=s.nontemporal)


def _shape_dict(s: TileShape) -> dict:
    return dict(tile_records=s.tile_records, slots=s.slots, pad_shift=s.pad_shift, wg_per_cu=s.wg_per_cu,
                order=s.order, nontemporal=s.nontemporal)


def tune_remap(ctx: Ctx, src_l: Layout, src, dst_l: Layout, dst, reps: int = 3, stream=None) -> dict:
    """Autotunes the pair's tile shape on these buffers (dst is overwritten)."""
    sp, sc = _dev(src)
    dp, dc = _dev(dst)
    best, bt, dt = TileShape(), ctypes.c_double(), ctypes.c_double()
    check(lib().adha_tune_remap(ctx.h, src_l.h, sp, sc, dst_l.h, dp, dc, reps, stream_ptr(stream),
                                ctypes.byref(best), ctypes.byref(bt), ctypes.byref(dt)))
    return dict(shape=_shape_dict(best), best_us=bt.value, default_us=dt.value)


def _items(items):
    arr = (RemapItem * max(1, len(items)))()
    for i, (sl, s, dl, d) in enumerate(items):
        sp, sc = _dev(s)
        dp, dc = _dev(d)
        arr[i] = RemapItem(sl.h.value, sp.value if sp else None, sc, dl.h.value, dp.value if dp else None, dc)
    return arr


def tune_batched(ctx: Ctx, items, reps: int = 3, stream=None) -> dict:
    arr = _items(items)
    tb, best, bt, dt = ctypes.c_uint32(), TileShape(), ctypes.c_double(), ctypes.c_double()
    check(lib().adha_tune_batched(ctx.h, len(items), arr, reps, stream_ptr(stream), ctypes.byref(tb),
                                  ctypes.byref(best), ctypes.byref(bt), ctypes.byref(dt)))
    return dict(tile_bytes=tb.value, shape=_shape_dict(best), best_us=bt.value, default_us=dt.value)


def tune_save(ctx: Ctx, path: str):
    check(lib().adha_tune_save(ctx.h, path.encode()))


def tune_load(ctx: Ctx, path: str):
    check(lib().adha_tune_load(ctx.h, path.encode()))


def describe(src_l: Layout, dst_l: Layout, cu_count: int = 256) -> dict:
    """Host-only description of a remap launch (tile shape, tiles, tail bytes)."""
    r = RemapInfo()
    check(lib().adha_remap_describe(src_l.h, dst_l.h, cu_count, ctypes.byref(r)))
    out = {k: getattr(r, k) for k, _ in RemapInfo._fields_ if k != "shape"}
    out.update(tile_records=r.shape.tile_records, slots=r.shape.slots, pad_shift=r.shape.pad_shift,
               wg_per_cu=r.shape.wg_per_cu, order=r.shape.order, nontemporal=r.shape.nontemporal)
    return out


def _host(a):
    """(pointer, capacity in bytes) of a host numpy array or CPU tensor (or (None, 0))."""
    if a is None:
        return None, 0
    if hasattr(a, "ctypes"):
        return ctypes.c_void_p(a.ctypes.data), a.nbytes
    return ctypes.c_void_p(a.data_ptr()), a.numel() * a.element_size()


def host_section_run(sec: Section, layout: Layout, buf, idx=None, table=None, threads: int = 0) -> int:
    """Runs a section on host memory; returns the number of out-of-range
    indices or keys met."""
    bp, bc = _host(buf)
    ip, ic = _host(idx)
    tp, tc = _host(table)
    bad = ctypes.c_uint64()
    check(lib().adha_host_section_run(sec.h, layout.h, bp, bc, ip, ic // 4, tp, tc, threads, ctypes.byref(bad)))
    return bad.value


def host_remap(src_l: Layout, src, dst_l: Layout, dst, threads: int = 0):
    sp, sc = _host(src)
    dp, dc = _host(dst)
    check(lib().adha_host_remap(src_l.h, sp, sc, dst_l.h, dp, dc, threads))


def section_run(ctx: Ctx, sec: Section, layout: Layout, buf, idx=None, stream=None):
    bp, bc = _dev(buf)
    ip, icap = _dev(idx)
    check(lib().adha_section_run(ctx.h, sec.h, layout.h, bp, bc, ip, icap // 4, stream_ptr(stream)))


def section_run_static(ctx: Ctx, sec: Section, layout: Layout, buf, idx=None, stream=None):
    """adha_section_run_static: the same run with no device allocation."""
    bp, bc = _dev(buf)
    ip, icap = _dev(idx)
    check(lib().adha_section_run_static(ctx.h, sec.h, layout.h, bp, bc, ip, icap // 4, stream_ptr(stream)))


def remap_in_place(ctx: Ctx, src_layout: Layout, dst_layout: Layout, buf, stream=None):
    """adha_remap_in_place: move, inside buf, the groups dst_layout does not
    share (same fields, tile and base) with src_layout."""
    bp, bc = _dev(buf)
    check(lib().adha_remap_in_place(ctx.h, src_layout.h, dst_layout.h, bp, bc, stream_ptr(stream)))


def plan_arena(plan: Plan):
    """(arena bytes, start layout, end layout) of a plan's placed execution;
    the layouts are borrowed from the plan."""
    b = ctypes.c_uint64()
    s, e = ctypes.c_void_p(), ctypes.c_void_p()
    check(lib().adha_plan_arena(plan.h, ctypes.byref(b), ctypes.byref(s), ctypes.byref(e)))
    return b.value, Layout(s, owned=False, keep=plan), Layout(e, owned=False, keep=plan)


def probe_stream(ctx: Ctx, kind: int, a, b, nbytes: int, reps: int = 5, stream=None) -> float:
    """adha_probe_stream: microseconds of a 16-byte read (0), write (1) or
    copy (2) stream over nbytes."""
    us = ctypes.c_double()
    ap, _ = _dev(a)
    bp, _ = _dev(b)
    check(lib().adha_probe_stream(ctx.h, kind, ap, bp, nbytes, reps, stream_ptr(stream), ctypes.byref(us)))
    return us.value


def probe_gather(ctx: Ctx, buf, stride: int, load_bytes: int, idx, out, reps: int = 5, stream=None) -> float:
    """adha_probe_gather: microseconds of one random load per index."""
    us = ctypes.c_double()
    bp, bc = _dev(buf)
    ip, icap = _dev(idx)
    op_, _ = _dev(out)
    check(lib().adha_probe_gather(ctx.h, bp, bc, stride, load_bytes, ip, icap // 4, op_, reps, stream_ptr(stream),
                                  ctypes.byref(us)))
    return us.value


def plan_placed(plan: Plan, i: int) -> Layout:
    """The plan's placed layout i (0: start; s + 1: section s), borrowed."""
    h = ctypes.c_void_p()
    check(lib().adha_plan_placed(plan.h, i, ctypes.byref(h)))
    return Layout(h, owned=False, keep=plan)


def run_placed(ctx: Ctx, plan: Plan, arena, idx=None, stream=None):
    """adha_run_placed: the plan in one buffer, data starting in the plan's
    start layout (plan_arena)."""
    ap, ac = _dev(arena)
    ip, icap = _dev(idx)
    check(lib().adha_run_placed(ctx.h, plan.h, ap, ac, ip, icap // 4, stream_ptr(stream)))


def run(ctx: Ctx, plan: Plan, in_layout: Layout, buf_a, buf_b, idx=None, stream=None):
    """Runs the plan; returns (final layout handle value, True if data ends in buf_b)."""
    ap, ac = _dev(buf_a)
    bp, bc = _dev(buf_b)
    cap = min(ac, bc) if buf_b is not None else ac
    ip, icap = _dev(idx)
    out_l = ctypes.c_void_p()
    in_b = ctypes.c_int32()
    check(lib().adha_run(ctx.h, plan.h, in_layout.h, ap, bp, cap, ip, icap // 4, stream_ptr(stream),
                         ctypes.byref(out_l), ctypes.byref(in_b)))
    return out_l.value, bool(in_b.value)


def run_flow(ctx: Ctx, plan: Plan, in_layout: Layout, buf_a, buf_b, taken, idx=None, stream=None):
    """Runs a structured program along the branch outcomes `taken` (one
    bool per branch); returns (final layout handle value, True if in b)."""
    ap, ac = _dev(buf_a)
    bp, bc = _dev(buf_b)
    ip, icap = _dev(idx)
    tk = (ctypes.c_uint8 * max(1, len(taken)))(*[1 if t else 0 for t in taken])
    out_l = ctypes.c_void_p()
    in_b = ctypes.c_int32()
    check(lib().adha_run_flow(ctx.h, plan.h, in_layout.h, ap, bp, min(ac, bc), ip, icap // 4, tk, len(taken),
                              stream_ptr(stream), ctypes.byref(out_l), ctypes.byref(in_b)))
    return out_l.value, bool(in_b.value)


def run_hetero(ctx: Ctx, plan: Plan, in_layout: Layout, in_device: int, dev_a, dev_b, host_a, host_b,
               idx_dev=None, idx_host=None, stream=None):
    """Runs a plan over both devices; returns (final layout handle value,
    final device 0/1, True if the data ends in buffer b)."""
    da, dac = _dev(dev_a)
    db, dbc = _dev(dev_b)
    ha, hac = _host(host_a)
    hb, hbc = _host(host_b)
    caps = [c for p, c in ((da, dac), (db, dbc), (ha, hac), (hb, hbc)) if p is not None]
    cap = min(caps) if caps else 0
    ip, ic = _dev(idx_dev)
    hp, hc = _host(idx_host)
    count = max(ic, hc) // 4
    if ip is not None and hp is not None:
        count = min(ic, hc) // 4
    out_l = ctypes.c_void_p()
    out_d = ctypes.c_int32()
    in_b = ctypes.c_int32()
    check(lib().adha_run_hetero(ctx.h, plan.h, in_layout.h, in_device, da, db, ha, hb, cap, ip, hp, count,
                                stream_ptr(stream), ctypes.byref(out_l), ctypes.byref(out_d), ctypes.byref(in_b)))
    return out_l.value, out_d.value, bool(in_b.value)


def mlp_forward(ctx: Ctx, params, x, y, stream=None):
    check(lib().adha_mlp_forward(ctx.h, params.data_ptr(), x.data_ptr(), x.shape[0], y.data_ptr(),
                                 stream_ptr(stream)))


def mlp_backward(ctx: Ctx, params, x, target, grad, loss=None, stream=None):
    check(lib().adha_mlp_backward(ctx.h, params.data_ptr(), x.data_ptr(), target.data_ptr(), x.shape[0],
                                  grad.data_ptr(), loss.data_ptr() if loss is not None else None,
                                  stream_ptr(stream)))


def mlp_adam(ctx: Ctx, params, grad, m, v, lr, b1, b2, eps, t, stream=None):
    check(lib().adha_mlp_adam(ctx.h, params.data_ptr(), grad.data_ptr(), m.data_ptr(), v.data_ptr(),
                              lr, b1, b2, eps, t, stream_ptr(stream)))


def train_opts(**kw) -> TrainOpts:
    o = TrainOpts()
    check(lib().adha_train_opts_default(ctypes.byref(o)))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def costmodel_train(ctx: Ctx, opts: TrainOpts = None) -> dict:
    opts = opts or train_opts()
    rep = TrainReport()
    check(lib().adha_costmodel_train(ctx.h, ctypes.byref(opts), ctypes.byref(rep)))
    return {k: getattr(rep, k) for k, _ in TrainReport._fields_}


def costmodel_save(ctx: Ctx, path: str):
    check(lib().adha_costmodel_save(ctx.h, path.encode()))


def costmodel_load(ctx: Ctx, path: str):
    check(lib().adha_costmodel_load(ctx.h, path.encode()))


def costmodel_predict(ctx: Ctx, sec: Section, layout: Layout) -> float:
    v = ctypes.c_double()
    check(lib().adha_costmodel_predict(ctx.h, sec.h, layout.h, ctypes.byref(v)))
    return v.value
