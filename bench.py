"""Benchmark of the layout-remap / section hot path on one MI355X.

One step = the three remaps of the single-remap workload on N = 2^26
records of 16 four-byte fields (64-byte records, 4 GiB per layout):
AoS -> SoA, SoA -> AoS and AoS -> AoSoA with groups {0-3}, {4-7}, {8-15}
tiled by 64 records.  `value` is the step's algorithmic bytes (each remap
reads and writes every record once: 2 * N * 64 bytes) over its time.

Besides the timed steps the run reports (outside the timed region):
  roofline      the remap kernel's achieved GB/s against 8 TB/s, from HIP
                events on the launch stream;
  cpu_baseline  the CPU oracle's remap on a bounded sample;
  program       the multi-section workload (N = 2^24, 32 fields, 8 sections,
                4 of them 16-neighbour gathers): program time under the
                planned layouts vs all-AoS and all-SoA, per-kernel GB/s;
  kmeans        the K-Means-shaped program (2^23 points, a direct loop and a
                per-cluster reduction of 32 features): planned vs all-AoS and
                all-SoA, per-section GB/s;
  medical       the Medical-shaped stencil program (256^3 image, 9 fields):
                planned vs all-AoS and all-SoA, per-section GB/s;
  flow          the multi-section workload with branches: expected time of
                the branch-aware plan vs a plan ignoring branches, all-AoS and
                all-SoA;
  subdword      remaps of structs with 1- and 2-byte fields (2^25 records,
                AoS <-> SoA, default shapes);
  hetero        plans over the GPU and the host (plain small program, data
                starting on the host, N = 2^10 .. 2^20): planned devices and
                run time vs all-GPU and all-host;
  batched       the 512-array batched remap: one graph launch vs one launch
                per array;
  learned       the learned cost model (the network kept in the package):
                planned program time with learned costs vs measured
                enumeration, over 64 seeded programs.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time
from concurrent.futures import ThreadPoolExecutor

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

# HBM traffic of one remap_tiles_kernel launch on this workload: rocprofv3
# --pmc FETCH_SIZE and WRITE_SIZE (KiB per dispatch, mean over the remap
# dispatches), each scaled by what the same counter reads for a plain 1 GiB
# device copy (fetch 524311.4 KiB, write 1048576 KiB).  It holds only for the
# kernel source it was taken on; any other source reports null.
REMAP_TRAFFIC = {"source_sha1": "2f60983d66d06b243a82110a7038279a7d756459",
                 "fetch_kib": 2097216.0, "write_kib": 4194322.5,
                 "copy_fetch_kib": 524311.5, "copy_write_kib": 1048576.0, "copy_bytes": 1 << 30}


def remap_traffic_bytes():
    import hashlib
    with open(os.path.join(ROOT, "paper_1407_4859_amd", "csrc", "remap.hip"), "rb") as f:
        if hashlib.sha1(f.read()).hexdigest() != REMAP_TRAFFIC["source_sha1"]:
            return None
    t = REMAP_TRAFFIC
    kib = t["copy_bytes"] / 1024.0
    return round((t["fetch_kib"] * kib / t["copy_fetch_kib"] + t["write_kib"] * kib / t["copy_write_kib"]) * 1024)


_T0 = time.perf_counter()


def log(*a):
    print("[bench %6.1fs]" % (time.perf_counter() - _T0), *a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--log2n", type=int, default=26, help="records of the single-remap workload")
    ap.add_argument("--program-log2n", type=int, default=24)
    ap.add_argument("--skip-program", action="store_true")
    ap.add_argument("--skip-batched", action="store_true")
    ap.add_argument("--skip-kmeans", action="store_true")
    ap.add_argument("--skip-hetero", action="store_true")
    ap.add_argument("--skip-flow", action="store_true")
    ap.add_argument("--skip-medical", action="store_true")
    ap.add_argument("--skip-subdword", action="store_true")
    ap.add_argument("--skip-probes", action="store_true")
    ap.add_argument("--only-subdword", action="store_true", help="the sub-dword remap leg only")
    ap.add_argument("--only-batched", action="store_true", help="the batched remap leg only")
    ap.add_argument("--cap-bytes", type=int, default=128, help="greedy grouping cap of the program leg's catalogue")
    ap.add_argument("--only-medical", action="store_true", help="the Medical-shaped stencil leg only")
    ap.add_argument("--only-medical-narrow", action="store_true",
                    help="the Medical-shaped leg with 1- and 2-byte image fields only")
    ap.add_argument("--skip-medical-narrow", action="store_true")
    ap.add_argument("--only-flow", action="store_true", help="the branching-program leg only")
    ap.add_argument("--only-hetero", action="store_true", help="the GPU + host planning leg only")
    ap.add_argument("--only-kmeans", action="store_true", help="the K-Means-shaped leg only (for profiling)")
    ap.add_argument("--skip-cpu", action="store_true")
    ap.add_argument("--skip-learned", action="store_true")
    ap.add_argument("--only-learned", action="store_true", help="skip everything but the cost-model leg")
    ap.add_argument("--train-model", action="store_true",
                    help="train a fresh network here instead of loading the packaged one")
    ap.add_argument("--train-samples", type=int, default=20000)
    ap.add_argument("--train-epochs", type=int, default=300)
    ap.add_argument("--programs", type=int, default=64)
    ap.add_argument("--learned-reps", type=int, default=1,
                    help="timed launches per (section, candidate) of the learned leg's measured enumeration")
    ap.add_argument("--program-seed0", type=int, default=1000)
    ap.add_argument("--save-model", default=None)
    ap.add_argument("--load-model", default=None)
    ap.add_argument("--only-remap", action="store_true", help="timed steps only (for profiling)")
    ap.add_argument("--only-probes", action="store_true", help="the bandwidth and random-access probes only")
    ap.add_argument("--only-program", action="store_true", help="the program leg only (for profiling)")
    ap.add_argument("--program-cost", choices=["measured", "analytic"], default="measured",
                    help="cost tables of the program leg's plan (analytic: no timing runs while planning)")
    ap.add_argument("--no-tune", action="store_true", help="use the default tile shapes")
    ap.add_argument("--save-tune", default=None, help="write the tuning database here after tuning")
    ap.add_argument("--load-tune", default=None, help="load a tuning database instead of tuning")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first copy 1 GiB with a plain device copy (scale for HBM byte counters)")
    return ap.parse_args()


def fill_fields(buf, spec, seed, torch, synth):
    """Write the seeded field values of every record into a device buffer,
    packed in field order (field f of record r at r * S + the sizes of the
    fields before f)."""
    n = spec.n
    S = spec.record_bytes
    view = buf[: n * S].view(n, S)
    chunk = 1 << 24
    off = 0
    for f, (dt, e) in enumerate(zip(spec.dtypes, spec.elem_bytes)):
        for s in range(0, n, chunk):
            c = min(chunk, n - s)
            z = synth.splitmix64_torch(seed, f, s, c, "cuda")
            view[s:s + c, off:off + e] = synth.decode_torch(z, dt, e)
        off += e


class Timer:
    """HIP-event timing on torch's current stream (the stream the library's
    kernels are launched on)."""

    def __init__(self, torch):
        self.torch = torch

    def time(self, fn, reps=5, warm=1):
        t = self.torch
        for _ in range(warm):
            fn()
        ts = []
        for _ in range(reps):
            a, b = t.cuda.Event(enable_timing=True), t.cuda.Event(enable_timing=True)
            a.record()
            fn()
            b.record()
            b.synchronize()
            ts.append(a.elapsed_time(b))
        ts.sort()
        return ts[len(ts) // 2], ts

    def time_cold(self, fn, reps=5, warm=1):
        """As time(), with a 512 MiB scratch buffer read before each timed
        launch (outside the events), so no launch finds its data in the
        256 MB last-level cache or the L2s from the one before.  The buffer
        is read, not written: evicting clean lines costs the timed launch no
        write-backs."""
        t = self.torch
        if getattr(self, "_flush", None) is None:
            self._flush = t.ones(1 << 26, dtype=t.int64, device="cuda")
        for _ in range(warm):
            fn()
        ts = []
        for r in range(reps):
            self._sink = self._flush.sum()
            a, b = t.cuda.Event(enable_timing=True), t.cuda.Event(enable_timing=True)
            a.record()
            fn()
            b.record()
            b.synchronize()
            ts.append(a.elapsed_time(b))
        ts.sort()
        return ts[len(ts) // 2], ts


# The measured ceilings of this run (set by the probes leg): copy and read
# stream rates in GB/s and the random-access rate in accesses per second.
CEIL = {}


def ceiling_fracs(alg_GBps, eff_GBps=None, gather=False):
    """A section's rate against the 8 TB/s peak and against the measured
    ceiling of its access pattern: the copy stream for a streamed pass, the
    random-access rate (128-byte lines) for a gather's effective bytes."""
    out = {"frac_of_peak": round(alg_GBps / HBM_PEAK_GBS, 4)}
    if gather:
        if CEIL.get("random_lines_GBps") and eff_GBps is not None:
            out["eff_frac_of_random_ceiling"] = round(eff_GBps / CEIL["random_lines_GBps"], 4)
    elif CEIL.get("copy_GBps"):
        out["frac_of_copy_ceiling"] = round(alg_GBps / CEIL["copy_GBps"], 4)
    return out


def cpu_baseline(synth):
    """The oracle's AoS -> SoA remap of the same struct (2^26 records),
    split over the host's cores by record ranges."""
    import oracle
    from oracle.layout import aos, soa
    n = 1 << 26
    spec = synth.config2_struct(n)
    eb = spec.elem_bytes
    La, Ls = aos(n, eb), soa(n, eb)
    rng = np.random.default_rng(2)
    src = rng.integers(0, 1 << 63, La.nbytes // 8, dtype=np.uint64).view(np.uint8)
    dst = np.zeros(Ls.nbytes, np.uint8)
    cores = os.cpu_count() or 1
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        pass
    sd, dd = np.ascontiguousarray(La.desc()), np.ascontiguousarray(Ls.desc())
    lib = oracle.lib()
    p = oracle._p
    bounds = [n * i // cores for i in range(cores + 1)]

    def part(i):
        lib.orc_remap(16, p(sd), p(src), p(dd), p(dst), bounds[i], bounds[i + 1])

    ts = []
    for _ in range(3):
        t0 = time.perf_counter()
        with ThreadPoolExecutor(cores) as ex:
            list(ex.map(part, range(cores)))
        ts.append(time.perf_counter() - t0)
    t = sorted(ts)[1]
    return {"value": round(2 * n * 64 / t / 1e9, 3), "unit": "GB/s", "cores": cores, "kind": "oracle",
            "sample": f"AoS->SoA remap of all 2^26 records x 64 B (8 GiB moved), median of 3, "
                      f"{cores} threads over record ranges; {t * 1e3:.0f} ms"}


def program_bench(A, synth, torch, timer, log2n, cost="measured", cap_bytes=64):
    n = 1 << log2n
    spec = synth.config3_struct(n)
    st = A.Struct.from_spec(spec)
    secs = synth.random_program(3, spec.n_fields)
    ss = [A.Section.from_spec(st, s) for s in secs]
    prog = A.Program(st, ss)
    aos_l, soa_l = A.Layout.aos(st), A.Layout.soa(st)
    idx = synth.uniform_index_torch(3, 999, n * 16, n, "cuda")
    ctx = A.Ctx(0)
    log("program: planning (%s costs)" % cost)
    t0 = time.perf_counter()
    src = A.COST_MEASURED if cost == "measured" else A.COST_ANALYTIC
    plan = A.Plan.create(ctx, prog, A.plan_opts(cost=src, catalogue=A.CAT_FULL, cap_bytes=cap_bytes, reps=3), idx=idx)
    plan_s = time.perf_counter() - t0
    analytic = A.Plan.create(ctx, prog, A.plan_opts(cost=A.COST_ANALYTIC, catalogue=A.CAT_FULL, cap_bytes=cap_bytes))
    # data that starts in AoS: the same tables solved with the entry remap charged
    fixed = plan.with_init(A.INIT_AOS)
    plans = {"adha": plan, "all_aos": A.Plan.uniform(prog, aos_l), "all_soa": A.Plan.uniform(prog, soa_l),
             "adha_analytic": analytic, "adha_from_aos": fixed}
    # every plan runs placed in one arena (only changed groups move)
    arena = torch.empty(max(A.plan_arena(p)[0] for p in plans.values()), dtype=torch.uint8, device="cuda")
    log("program: filling", n, "records; arena", arena.numel(), "bytes")
    fill_fields(arena, spec, 3, torch, synth)
    out = {"workload": f"N=2^{log2n} records, 32 fields (20 f32, 8 i32, 4 f64; 144 B), 8 GEN sections "
                       f"(seed 3), 4 gathering 16 uniform neighbours",
           "candidates": plan.n_candidates, "cap_bytes": cap_bytes, "plan_seconds": round(plan_s, 2),
           "executor": "placed in one arena; a remap moves only the groups that change"}
    for name, pl in plans.items():
        def go(pl=pl):
            A.run_placed(ctx, pl, arena, idx)
        ms, _ = timer.time(go, reps=5, warm=1)
        out[name + "_ms"] = round(ms, 3)
        out[name + "_choices"] = pl.choices()
        out[name + "_arena_bytes"] = A.plan_arena(pl)[0]
    ctx.check()
    best_base = min(out["all_aos_ms"], out["all_soa_ms"])
    out["speedup_vs_best_uniform"] = round(best_base / out["adha_ms"], 3)
    out["adha_beats_both"] = out["adha_ms"] < best_base
    out["predicted_adha_ms"] = round(plan.cost / 1e3, 3)
    # remap costs by pair: the measured table against the bytes each pair moves
    T, R = plan.tables()
    C = plan.n_candidates
    offd = [R[a][b] for a in range(C) for b in range(C) if a != b and R[a][b] > 0]
    out["remap_table_us"] = {"pairs": len(offd), "min": round(min(offd), 1), "median": round(sorted(offd)[len(offd) // 2], 1),
                             "max": round(max(offd), 1), "aos_to_soa": round(R[0][1], 1)}
    # data born in AoS (the entry remap charged): ADHA vs all-AoS vs all-SoA
    # with the entry remap
    soa_entry = A.Plan.uniform(prog, soa_l).with_init(A.INIT_AOS)
    ms_soa_entry, _ = timer.time(lambda: A.run_placed(ctx, soa_entry, arena, idx), reps=5, warm=1)
    out["from_aos"] = {"adha_ms": out["adha_from_aos_ms"], "all_aos_ms": out["all_aos_ms"],
                       "all_soa_with_entry_remap_ms": round(ms_soa_entry, 3),
                       "adha_choices": fixed.choices(), "predicted_adha_ms": round(fixed.cost / 1e3, 3)}
    out["from_aos"]["speedup_vs_best_uniform"] = round(
        min(out["all_aos_ms"], ms_soa_entry) / out["adha_from_aos_ms"], 3)
    # per-section kernel time under the chosen layouts (HIP events around
    # each launch; timings do not depend on the buffer's values)
    per = []
    for s, (sec, c) in enumerate(zip(ss, plan.choices())):
        lay = plan.candidate(c)
        ms, _ = timer.time_cold(lambda: A.section_run(ctx, sec, lay, arena, idx if secs[s].degree else None),
                                reps=7, warm=1)
        t_us = ms * 1e3
        alg = sec.bytes / (t_us * 1e3)
        eff = sec.effective_bytes(lay) / (t_us * 1e3)
        per.append({"section": s, "degree": secs[s].degree, "read": len(secs[s].read),
                    "write": len(secs[s].write), "layout": c, "us": round(t_us, 1),
                    "alg_GBps": round(alg, 1), "eff_GBps": round(eff, 1),
                    **ceiling_fracs(alg, eff, gather=secs[s].degree > 0)})
    ctx.check()
    out["sections"] = per
    return out


def kmeans_bench(A, synth, torch, timer, log2n=23):
    """The K-Means-shaped program: a direct loop over 32 features, then a
    reduction of the features per cluster (5 keys), planned with measured
    costs and compared with all-AoS and all-SoA."""
    n = 1 << log2n
    spec = synth.kmeans_struct(n)
    st = A.Struct.from_spec(spec)
    gen_spec, (rd, key, nk) = synth.kmeans_sections()
    out = torch.zeros(nk * (len(rd) + 1) * 8, dtype=torch.uint8, device="cuda")
    gen = A.Section.from_spec(st, gen_spec)
    red = A.Section.reduce(st, rd, key, nk, out)
    prog = A.Program(st, [gen, red])
    aos_l, soa_l = A.Layout.aos(st), A.Layout.soa(st)
    cap = max(aos_l.nbytes, soa_l.nbytes) + (1 << 26)
    src = torch.empty(aos_l.nbytes, dtype=torch.uint8, device="cuda")
    buf_a = torch.empty(cap, dtype=torch.uint8, device="cuda")
    buf_b = torch.empty(cap, dtype=torch.uint8, device="cuda")
    log("kmeans: filling", n, "records")
    fill_fields(src, spec, 6, torch, synth)
    keys = synth.uniform_index_torch(6, 77, n, nk, "cuda")
    src[: n * spec.record_bytes].view(n, spec.record_bytes)[:, 4 * key:4 * key + 4] = \
        keys.view(torch.uint8).view(n, 4)
    ctx = A.Ctx(0)

    def load(lay):
        """buf_a holds the points in layout `lay` (the keys must be valid)."""
        if lay.equals(aos_l):
            buf_a[: aos_l.nbytes].copy_(src)
        else:
            A.remap(ctx, aos_l, src, lay, buf_a)

    t0 = time.perf_counter()
    plan = A.Plan.create(ctx, prog, A.plan_opts(cost=A.COST_MEASURED, catalogue=A.CAT_FULL, cap_bytes=64, reps=3))
    plan_s = time.perf_counter() - t0
    res = {"workload": f"N=2^{log2n} points, 32 f32 features + i32 cluster key (5 clusters) + f32 result "
                       f"(136 B); GEN over the features, then their per-cluster reduction",
           "candidates": plan.n_candidates, "plan_seconds": round(plan_s, 2)}
    for name, pl in (("adha", plan), ("all_aos", A.Plan.uniform(prog, aos_l)),
                     ("all_soa", A.Plan.uniform(prog, soa_l))):
        first = pl.candidate(pl.choices()[0])
        load(first)      # runs start from the plan's first layout and leave buf_a's keys as they are
        ms = back_to_back_ms(timer, lambda: A.run(ctx, pl, first, buf_a, buf_b))
        res[name + "_ms"] = round(ms, 3)
        res[name + "_choices"] = pl.choices()
    ctx.check()
    res["speedup_vs_best_uniform"] = round(min(res["all_aos_ms"], res["all_soa_ms"]) / res["adha_ms"], 3)
    per = []
    for s, sec in enumerate((gen, red)):
        for lname, lay in (("planned", plan.candidate(plan.choices()[s])), ("aos", aos_l), ("soa", soa_l)):
            load(lay)
            ms, _ = timer.time_cold(lambda: A.section_run(ctx, sec, lay, buf_a), reps=7, warm=1)
            alg = sec.bytes / (ms * 1e6)
            per.append({"section": s, "layout": lname, "us": round(ms * 1e3, 1),
                        "alg_GBps": round(alg, 1), **ceiling_fracs(alg)})
    ctx.check()
    res["sections"] = per
    return res


def medical_bench(A, synth, torch, timer, side=256, narrow=False):
    """The Medical-shaped program on a side^3 image of 9 f32 fields (narrow:
    V1-V3 U16, U1-U3 F32, S U8, T I16, interpT F32): two 7-point stencils and
    two direct loops, planned with measured costs and compared with all-AoS
    and all-SoA; per-section times and GB/s."""
    spec = synth.medical_narrow_struct(side) if narrow else synth.medical_struct(side)
    n = spec.n
    st = A.Struct.from_spec(spec)
    grid = (side, side, side)
    ss = []
    for rd, wr, offs in synth.medical_sections():
        ss.append(A.Section.stencil(st, rd, wr, grid, offs) if offs else A.Section(st, A.OP_GEN, rd, wr, 0))
    prog = A.Program(st, ss)
    aos_l, soa_l = A.Layout.aos(st), A.Layout.soa(st)
    cap = max(aos_l.nbytes, soa_l.nbytes) + (1 << 24)
    buf_a = torch.empty(cap, dtype=torch.uint8, device="cuda")
    buf_b = torch.empty(cap, dtype=torch.uint8, device="cuda")
    fill_fields(buf_a, spec, 13, torch, synth)
    ctx = A.Ctx(0)
    t0 = time.perf_counter()
    plan = A.Plan.create(ctx, prog, A.plan_opts(cost=A.COST_MEASURED, catalogue=A.CAT_FULL, cap_bytes=64, reps=3))
    plan_s = time.perf_counter() - t0
    fields = ("V1-V3 u16, U1-U3 f32, S u8, T i16, interpT f32 (18 B)" if narrow else "9 f32 fields (36 B)")
    res = {"workload": f"{side}^3 image, {fields}; 7-point stencil U->V1, direct V1,S,T->interpT, "
                       f"7-point stencil V->U1, direct U,interpT->V2,V3",
           "candidates": plan.n_candidates, "plan_seconds": round(plan_s, 2)}
    for name, pl in (("adha", plan), ("all_aos", A.Plan.uniform(prog, aos_l)), ("all_soa", A.Plan.uniform(prog, soa_l))):
        first = pl.candidate(pl.choices()[0])
        ms = back_to_back_ms(timer, lambda: A.run(ctx, pl, first, buf_a, buf_b))
        res[name + "_ms"] = round(ms, 3)
        res[name + "_choices"] = pl.choices()
    ctx.check()
    res["speedup_vs_best_uniform"] = round(min(res["all_aos_ms"], res["all_soa_ms"]) / res["adha_ms"], 3)
    per = []
    for s, (sec, c) in enumerate(zip(ss, plan.choices())):
        for lname, lay in (("planned", plan.candidate(c)), ("aos", aos_l), ("soa", soa_l)):
            ms, _ = timer.time_cold(lambda: A.section_run(ctx, sec, lay, buf_a), reps=7, warm=1)
            alg = sec.bytes / (ms * 1e6)
            per.append({"section": s, "stencil": sec.degree > 0, "layout": lname, "us": round(ms * 1e3, 1),
                        "alg_GBps": round(alg, 1),
                        "eff_GBps": round(sec.effective_bytes(lay) / (ms * 1e6), 1), **ceiling_fracs(alg)})
    ctx.check()
    res["sections"] = per
    return res


FLOW_TOKENS = [0, 1, -1, 2, 3, -2, 4, -3, 5, -1, 6, -3, 7]   # IF = -1, ELSE = -2, END = -3
FLOW_PROBS = [0.6, 0.3]


def flow_bench(A, synth, torch, timer, log2n=24):
    """The multi-section workload with branches: sections 2-3 run with
    probability 0.6, else section 4; section 6 with probability 0.3.  The
    expected time over the four outcomes for the branch-aware plan, the plan
    made as if every section ran in sequence, all-AoS and all-SoA."""
    import itertools
    n = 1 << log2n
    spec = synth.config3_struct(n)
    st = A.Struct.from_spec(spec)
    secs = synth.random_program(3, spec.n_fields)
    ss = [A.Section.from_spec(st, s) for s in secs]
    linear = A.Program(st, ss)
    prog = A.Program(st, ss)
    prog.set_flow(FLOW_TOKENS, FLOW_PROBS)
    aos_l, soa_l = A.Layout.aos(st), A.Layout.soa(st)
    cap = max(aos_l.nbytes, soa_l.nbytes) + (1 << 26)
    buf_a = torch.empty(cap, dtype=torch.uint8, device="cuda")
    buf_b = torch.empty(cap, dtype=torch.uint8, device="cuda")
    fill_fields(buf_a, spec, 3, torch, synth)
    idx = synth.uniform_index_torch(3, 999, n * 16, n, "cuda")
    ctx = A.Ctx(0)
    t0 = time.perf_counter()
    plan = A.Plan.create(ctx, prog, A.plan_opts(cost=A.COST_MEASURED, catalogue=A.CAT_FULL, cap_bytes=64, reps=3),
                         idx=idx)
    plan_s = time.perf_counter() - t0
    lin = A.Plan.create(ctx, linear, A.plan_opts(cost=A.COST_MEASURED, catalogue=A.CAT_FULL, cap_bytes=64, reps=3),
                        idx=idx)
    blind = A.Plan.explicit(prog, [lin.candidate(c) for c in lin.choices()])
    plans = {"adha_flow": plan, "adha_ignoring_branches": blind, "all_aos": A.Plan.uniform(prog, aos_l),
             "all_soa": A.Plan.uniform(prog, soa_l)}
    res = {"workload": f"N=2^{log2n} records, the 8-section program (seed 3) with branches: "
                       f"0 1 IF(0.6) 2 3 ELSE 4 END 5 IF(0.3) 6 END 7",
           "plan_seconds": round(plan_s, 2), "adha_flow_choices": plan.choices(), "adha_flow_joins": plan.joins(2),
           "predicted_expected_ms": round(plan.cost / 1e3, 3), "outcomes": {}}
    for name, pl in plans.items():
        first = pl.candidate(pl.choices()[0])
        exp_ms = 0.0
        for taken in itertools.product([1, 0], repeat=2):
            prob = 1.0
            for p, t in zip(FLOW_PROBS, taken):
                prob *= p if t else 1.0 - p
            ms, _ = timer.time(lambda: A.run_flow(ctx, pl, first, buf_a, buf_b, taken, idx), reps=3, warm=1)
            res["outcomes"].setdefault(name, {})["".join(map(str, taken))] = round(ms, 3)
            exp_ms += prob * ms
        res[name + "_expected_ms"] = round(exp_ms, 3)
    ctx.check()
    best_uniform = min(res["all_aos_expected_ms"], res["all_soa_expected_ms"])
    res["speedup_vs_best_uniform"] = round(best_uniform / res["adha_flow_expected_ms"], 3)
    res["gain_vs_ignoring_branches"] = round(res["adha_ignoring_branches_expected_ms"] /
                                             res["adha_flow_expected_ms"], 3)

    # Other branch probabilities on the same measured tables: the predicted
    # expected cost of the branch-aware plan (the library's solver) against
    # that of the plan that ignores branches, then the setting with the
    # largest predicted gain planned and measured like the default one.
    T, R = plan.tables()
    cands = [plan.candidate(c) for c in range(plan.n_candidates)]
    blind_nodes = [next(i for i, L in enumerate(cands) if L.equals(lin.candidate(c))) for c in lin.choices()]

    def blind_expected(probs):
        total = 0.0
        for taken in itertools.product([1, 0], repeat=2):
            prob = 1.0
            for p, t in zip(probs, taken):
                prob *= p if t else 1.0 - p
            path = [0, 1] + ([2, 3] if taken[0] else [4]) + [5] + ([6] if taken[1] else []) + [7]
            c = [blind_nodes[s] for s in path]
            cost = sum(T[s][blind_nodes[s]] for s in path) + sum(R[a][b] for a, b in zip(c, c[1:]))
            total += prob * cost
        return total

    sweep = []
    for p1 in (0.05, 0.2, 0.5, 0.8, 0.95):
        for p2 in (0.05, 0.2, 0.5, 0.8, 0.95):
            aware = A.flow_solve(T, R, FLOW_TOKENS, [p1, p2])[0]
            sweep.append((blind_expected([p1, p2]) / aware, p1, p2))
    sweep.sort(reverse=True)
    g, p1, p2 = sweep[0]
    res["probability_sweep"] = {"predicted_gain_max": round(g, 3), "at": [p1, p2],
                                "predicted_gain_min": round(sweep[-1][0], 3)}
    if g > 1.01:
        prog2 = A.Program(st, ss)
        prog2.set_flow(FLOW_TOKENS, [p1, p2])
        log("flow: planning at probabilities", p1, p2)
        plan2 = A.Plan.create(ctx, prog2, A.plan_opts(cost=A.COST_MEASURED, catalogue=A.CAT_FULL, cap_bytes=64,
                                                      reps=3), idx=idx)
        blind2 = A.Plan.explicit(prog2, [lin.candidate(c) for c in lin.choices()])
        measured = {}
        for name, pl in (("adha_flow", plan2), ("adha_ignoring_branches", blind2)):
            first = pl.candidate(pl.choices()[0])
            exp_ms = 0.0
            for taken in itertools.product([1, 0], repeat=2):
                prob = 1.0
                for p, t in zip((p1, p2), taken):
                    prob *= p if t else 1.0 - p
                ms, _ = timer.time(lambda: A.run_flow(ctx, pl, first, buf_a, buf_b, taken, idx), reps=3, warm=1)
                exp_ms += prob * ms
            measured[name + "_expected_ms"] = round(exp_ms, 3)
        ctx.check()
        measured["predicted_expected_ms"] = round(plan2.cost / 1e3, 3)
        measured["measured_gain"] = round(measured["adha_ignoring_branches_expected_ms"] /
                                          measured["adha_flow_expected_ms"], 3)
        res["probability_sweep"]["measured_at_max"] = measured
    return res


def hetero_bench(A, synth, torch):
    """Plans over the GPU and the host for the plain small program (8 f32
    fields, MULADD3, SUB2, SUM) with its data starting in AoS on the host,
    for N = 2^10 .. 2^20: the planned devices, and the wall time of the
    planned run against all-GPU (which first copies the data over) and
    all-host runs."""
    ctx = A.Ctx(0)
    rows = []
    for log2n in (10, 12, 14, 16, 18, 20):
        n = 1 << log2n
        spec = synth.config1_struct(n)
        st = A.Struct.from_spec(spec)
        prog = A.Program(st, [A.Section.from_spec(st, s) for s in synth.config1_sections()])
        aos = A.Layout.aos(st)
        img = synth.pack_aos(synth.record_matrix(1, n, spec.dtypes, spec.elem_bytes), n).reshape(-1)
        cap = max(aos.nbytes, A.Layout.soa(st).nbytes) + 4096
        dev = [torch.empty(cap, dtype=torch.uint8, device="cuda") for _ in range(2)]
        hst = [torch.empty(cap, dtype=torch.uint8).pin_memory() for _ in range(2)]
        src = torch.from_numpy(img)
        t0 = time.perf_counter()
        plan = A.Plan.create(ctx, prog, A.plan_opts(cost=A.COST_MEASURED, catalogue=A.CAT_FULL, reps=5,
                                                    devices=A.DEVICES_GPU_HOST, init=A.INIT_HOST_AOS))
        plan_s = time.perf_counter() - t0
        gpu = A.Plan.create(ctx, prog, A.plan_opts(cost=A.COST_MEASURED, catalogue=A.CAT_FULL, reps=5))
        host_only = A.Plan.explicit(prog, [aos] * 3, [1] * 3)

        def timed(pl):
            ts = []
            for r in range(6):
                hst[0][: img.size].copy_(src)
                torch.cuda.synchronize()
                t = time.perf_counter()
                A.run_hetero(ctx, pl, aos, 1, dev[0], dev[1], hst[0], hst[1])
                torch.cuda.synchronize()
                if r:
                    ts.append((time.perf_counter() - t) * 1e6)
            return sorted(ts)[len(ts) // 2]

        row = {"log2n": log2n, "devices": plan.devices(), "choices": plan.choices(),
               "predicted_us": round(plan.cost, 1), "plan_s": round(plan_s, 2),
               "planned_us": round(timed(plan), 1), "all_gpu_us": round(timed(gpu), 1),
               "all_host_us": round(timed(host_only), 1)}
        best = min(row["all_gpu_us"], row["all_host_us"])
        row["planned_vs_best_single_device"] = round(row["planned_us"] / best, 3)
        ctx.check()
        rows.append(row)
        log("hetero:", row)
    return {"workload": "plain small program (8 f32, MULADD3, SUB2, SUM), data starting in AoS on the host, "
                        "N = 2^10 .. 2^20; host threads: %s" % (os.cpu_count(),), "rows": rows}


def batched_bench(A, synth, torch, timer):
    arrs = synth.config4_arrays()
    ctx = A.Ctx(0)
    items, keep = [], []
    total = 0
    log("batched: allocating", len(arrs), "arrays")
    for a in arrs:
        st = A.Struct(a["n"], [A.RAW] * len(a["elem_bytes"]), a["elem_bytes"])
        la = A.Layout.aos(st)
        lb = A.Layout.create(st, a["target_gof"], a["target_tiles"])
        src = torch.empty(la.nbytes, dtype=torch.uint8, device="cuda")
        src.random_(0, 256)
        dst = torch.empty(lb.nbytes, dtype=torch.uint8, device="cuda")
        items.append((la, src, lb, dst))
        keep.append(st)
        total += 2 * a["n"] * sum(a["elem_bytes"])
    batch = A.BatchItems(items)          # marshalled once, as a C caller would
    log("batched: tuning the batch policy")
    tuned = A.tune_batched(ctx, items, reps=3)   # untimed; keeps the fastest policy in the context
    g_ms, _ = timer.time(lambda: A.remap_batched(ctx, batch, A.BATCH_GRAPH), reps=5, warm=2)
    b_ms, _ = timer.time(lambda: A.remap_batched(ctx, batch, 0), reps=5, warm=1)
    s_ms, _ = timer.time(lambda: A.remap_batched(ctx, batch, A.BATCH_SEPARATE), reps=5, warm=1)
    ctx.check()
    return {"workload": "512 arrays, N log-uniform in [2^10, 2^22], 4-24 fields of 4 or 8 bytes, AoS -> SoA "
                        "or AoSoA (groups of 2-8, 64-record tiles), seed 4",
            "algorithmic_bytes": total, "tuned_policy": {"tile_bytes": tuned["tile_bytes"], **tuned["shape"]},
            "tuned_persistent_ms": round(tuned["best_us"] / 1e3, 3),
            "default_policy_persistent_ms": round(tuned["default_us"] / 1e3, 3),
            "graph_ms": round(g_ms, 3), "persistent_ms": round(b_ms, 3),
            "separate_launches_ms": round(s_ms, 3), "graph_GBps": round(total / g_ms / 1e6, 1),
            "separate_GBps": round(total / s_ms / 1e6, 1),
            "graph_frac_of_peak": round(total / g_ms / 1e6 / HBM_PEAK_GBS, 3)}


def probes_bench(A, synth, torch):
    """The ceilings: plain 16-byte read, write and copy streams over 4 GiB,
    and random single loads (the access of a gather's neighbour field) into
    a 2.4 GB buffer -- the program workload's AoS size -- at several record
    strides and load widths, 2^26 accesses each."""
    ctx = A.Ctx(0)
    nbytes = 1 << 32
    a = torch.ones(nbytes, dtype=torch.uint8, device="cuda")
    b = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    out = {"stream_bytes": nbytes}
    for kind, name in ((0, "read"), (1, "write"), (2, "copy")):
        us = A.probe_stream(ctx, kind, a, b, nbytes, reps=5)
        moved = 2 * nbytes if kind == 2 else nbytes
        out[name + "_GBps"] = round(moved / us / 1e3, 1)
        out[name + "_frac_of_peak"] = round(moved / us / 1e3 / HBM_PEAK_GBS, 3)
    del b
    buf_bytes = (1 << 24) * 144
    n = 1 << 26
    res = torch.empty(n * 4, dtype=torch.uint8, device="cuda")
    rows = []
    for stride, lb in ((4, 4), (16, 16), (64, 4), (64, 16), (64, 64), (128, 4), (128, 64), (128, 128),
                       (144, 4), (144, 16)):
        records = buf_bytes // stride
        idx = synth.uniform_index_torch(9, stride, n, records, "cuda")
        us = A.probe_gather(ctx, a[:buf_bytes], stride, lb, idx, res, reps=5)
        rate = n / us * 1e6
        rows.append({"stride": stride, "load_bytes": lb, "us": round(us, 1), "G_accesses_per_s": round(rate / 1e9, 2),
                     "GBps_at_64B_per_access": round(rate * 64 / 1e9, 1),
                     "GBps_at_128B_per_access": round(rate * 128 / 1e9, 1)})
        del idx
    ctx.check()
    out["random_access"] = {"buffer_bytes": buf_bytes, "accesses": n, "rows": rows}
    return out


def back_to_back_ms(timer, fn, inner=10, reps=5):
    """Milliseconds per call of fn over `inner` calls between two events:
    for programs of a few hundred microseconds the host work of one call
    then overlaps the GPU work of the previous one, as in a loop."""
    ms, _ = timer.time(lambda: [fn() for _ in range(inner)], reps=reps, warm=1)
    return ms / inner


def subdword_bench(A, torch, timer, log2n=25):
    """Remaps of structs with 1- and 2-byte fields (the tile kernel's byte
    mode), default tile shapes, AoS <-> SoA."""
    n = 1 << log2n
    out = {"workload": "N=2^%d records; AoS->SoA and SoA->AoS with default shapes" % log2n}
    ctx = A.Ctx(0)
    for name, eb in (("8x1B+4x2B+4x4B", [1] * 8 + [2] * 4 + [4] * 4), ("8x2B+8x4B", [2] * 8 + [4] * 8),
                     ("24x1B", [1] * 24)):
        st = A.Struct(n, [A.RAW] * len(eb), eb)
        La, Ls = A.Layout.aos(st), A.Layout.soa(st)
        a = torch.empty(La.nbytes, dtype=torch.uint8, device="cuda").random_(0, 256)
        b = torch.empty(Ls.nbytes, dtype=torch.uint8, device="cuda")
        moved = 2 * n * sum(eb)
        row = {"record_bytes": sum(eb), "shape": A.get_shape(ctx, La, Ls)}
        for d, fn in (("aos_to_soa", lambda: A.remap(ctx, La, a, Ls, b)),
                      ("soa_to_aos", lambda: A.remap(ctx, Ls, b, La, a))):
            ms, _ = timer.time(fn, reps=7, warm=1)
            row[d] = {"ms": round(ms, 4), "GBps": round(moved / ms / 1e6, 1),
                      "frac": round(moved / ms / 1e6 / HBM_PEAK_GBS, 4)}
        out[name] = row
        del a, b
    ctx.check()
    return out


def path_cost(T, R, path):
    """Cost of a layout choice per section under tables T (k x C) and R (C x C)."""
    c = T[0][path[0]]
    for s in range(1, len(path)):
        c += R[path[s - 1]][path[s]] + T[s][path[s]]
    return c


def learned_bench(A, synth, torch, args):
    """Plans seeded 8-section programs with learned, analytic and measured
    costs; each plan is scored under the measured tables (the enumeration's
    ground truth).  The network is the one kept in the package (trained on
    this kind of device by train_costmodel.py), unless --train-model asks for
    a fresh one.  All three planners price remaps alike: one measured
    whole-struct remap scaled by the bytes each pair moves."""
    ctx = A.Ctx(0)
    if not args.train_model:
        path = args.load_model or A.DEFAULT_MODEL
        A.costmodel_load(ctx, path)
        rep = {"loaded": os.path.relpath(path, os.path.dirname(os.path.abspath(__file__)))}
        meta = os.path.splitext(path)[0] + ".json"
        if os.path.exists(meta):
            with open(meta) as fh:
                rep["trained"] = json.load(fh)
    else:
        log("learned: generating and timing", args.train_samples, "sections")
        rep = A.costmodel_train(ctx, A.train_opts(n_samples=args.train_samples, epochs=args.train_epochs,
                                                  min_log2_n=16, max_log2_n=24, reps=3,
                                                  progress_every=1000))
        rep = {k: (round(v, 4) if isinstance(v, float) else v) for k, v in rep.items()}
        if args.save_model:
            A.costmodel_save(ctx, args.save_model)
    rows = []
    for seed in range(args.program_seed0, args.program_seed0 + args.programs):
        z = synth.splitmix64(5, seed, 0, 1)
        n = 1 << (20 + int(((int(z[0]) >> 32) * 5) >> 32))
        spec = synth.config3_struct(n)
        st = A.Struct.from_spec(spec)
        ss = [A.Section.from_spec(st, s) for s in synth.random_program(seed % 256, 32)]
        prog = A.Program(st, ss)
        idx = synth.uniform_index_torch(seed % 256, 999, n * 16, n, "cuda")
        # the enumeration's ground truth: every (section, candidate) timed
        # (one warm-up launch, then one timed launch)
        pl_m = A.Plan.create(ctx, prog, A.plan_opts(cost=A.COST_MEASURED, reps=args.learned_reps, pair_remaps=0),
                             idx=idx)
        pl_l = A.Plan.create(ctx, prog, A.plan_opts(cost=A.COST_LEARNED), idx=idx)
        # the network's pick verified on the device: the sections of the
        # chosen path timed, then solved again (a few rounds)
        pl_v = A.Plan.create(ctx, prog, A.plan_opts(cost=A.COST_LEARNED, verify_rounds=4, reps=1), idx=idx)
        pl_a = A.Plan.create(ctx, prog, A.plan_opts(cost=A.COST_ANALYTIC))
        T, R = pl_m.tables()
        # without the network: analytic section costs, same measured remap costs
        Ta, _ = pl_a.tables()
        _, a_path = A.pdl_solve(Ta, R)
        rows.append(dict(seed=seed, log2n=n.bit_length() - 1, measured_us=round(pl_m.cost, 1),
                         learned_ratio=round(path_cost(T, R, pl_l.choices()) / pl_m.cost, 4),
                         verified_ratio=round(path_cost(T, R, pl_v.choices()) / pl_m.cost, 4),
                         verified_entries=pl_v.verified, plan_s_verified=round(pl_v.seconds, 3),
                         analytic_ratio=round(path_cost(T, R, a_path) / pl_m.cost, 4),
                         plan_s_measured=round(pl_m.seconds, 3), plan_s_learned=round(pl_l.seconds, 4)))
        log("learned:", rows[-1])
        del idx
        torch.cuda.empty_cache()
    lr = [r["learned_ratio"] for r in rows]
    ar = [r["analytic_ratio"] for r in rows]
    return {"workload": "%d seeded programs (seeds %d..%d) of 8 sections on the 32-field struct, N = 2^20..2^24; "
                        "ratio = program time of the plan / measured-enumeration optimum, under the measured tables"
                        % (len(rows), args.program_seed0, args.program_seed0 + args.programs - 1),
            "model": rep, "programs": len(rows),
            "gate_mean_ratio": 1.05, "gate_met": bool(np.mean(lr) <= 1.05),
            "learned_mean_ratio": round(float(np.mean(lr)), 4), "learned_max_ratio": round(float(np.max(lr)), 4),
            "verified_mean_ratio": round(float(np.mean([r["verified_ratio"] for r in rows])), 4),
            "verified_max_ratio": round(float(np.max([r["verified_ratio"] for r in rows])), 4),
            "verified_entries_mean": round(float(np.mean([r["verified_entries"] for r in rows])), 1),
            "plan_seconds_verified": round(sum(r["plan_s_verified"] for r in rows), 2),
            "analytic_mean_ratio": round(float(np.mean(ar)), 4), "analytic_max_ratio": round(float(np.max(ar)), 4),
            "plan_seconds_measured": round(sum(r["plan_s_measured"] for r in rows), 2),
            "plan_seconds_learned": round(sum(r["plan_s_learned"] for r in rows), 3),
            "plan_time_ratio_measured_over_learned": round(
                sum(r["plan_s_measured"] for r in rows) / max(1e-9, sum(r["plan_s_learned"] for r in rows)), 1),
            "rows": rows}


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU design is "
              "documented but not built", file=sys.stderr)
        sys.exit(2)
    import torch
    from paper_1407_4859_amd import adha as A
    from paper_1407_4859_amd import synth

    if not torch.cuda.is_available():
        print("no GPU visible", file=sys.stderr)
        sys.exit(1)
    timer = Timer(torch)
    if args.only_learned:
        print(json.dumps({"learned": learned_bench(A, synth, torch, args)}), flush=True)
        return
    if args.only_probes:
        print(json.dumps({"probes": probes_bench(A, synth, torch)}), flush=True)
        return
    if args.only_medical:
        print(json.dumps({"medical": medical_bench(A, synth, torch, timer)}), flush=True)
        return
    if args.only_medical_narrow:
        print(json.dumps({"medical_narrow": medical_bench(A, synth, torch, timer, narrow=True)}), flush=True)
        return
    if args.only_batched:
        print(json.dumps({"batched": batched_bench(A, synth, torch, timer)}), flush=True)
        return
    if args.only_subdword:
        print(json.dumps({"subdword": subdword_bench(A, torch, timer)}), flush=True)
        return
    if args.only_flow:
        print(json.dumps({"flow": flow_bench(A, synth, torch, timer, args.program_log2n)}), flush=True)
        return
    if args.only_hetero:
        print(json.dumps({"hetero": hetero_bench(A, synth, torch)}), flush=True)
        return
    if args.only_kmeans:
        print(json.dumps({"kmeans": kmeans_bench(A, synth, torch, timer)}), flush=True)
        return
    if args.only_program:
        print(json.dumps({"program": program_bench(A, synth, torch, timer, args.program_log2n, args.program_cost,
                                                   args.cap_bytes)}),
              flush=True)
        return
    n = 1 << args.log2n
    spec = synth.config2_struct(n)
    st = A.Struct.from_spec(spec)
    gof, tiles = synth.config2_aosoa()
    La, Ls, Lt = A.Layout.aos(st), A.Layout.soa(st), A.Layout.create(st, gof, tiles)
    ctx = A.Ctx(0)
    log("single remap: filling", n, "records")
    a = torch.empty(La.nbytes, dtype=torch.uint8, device="cuda")
    fill_fields(a, spec, 2, torch, synth)
    s = torch.empty(Ls.nbytes, dtype=torch.uint8, device="cuda")
    t = torch.empty(Lt.nbytes, dtype=torch.uint8, device="cuda")
    b = torch.empty(La.nbytes, dtype=torch.uint8, device="cuda")
    pairs = [("aos_to_soa", La, a, Ls, s), ("soa_to_aos", Ls, s, La, b), ("aos_to_aosoa", La, a, Lt, t)]
    step_bytes = 3 * 2 * n * spec.record_bytes

    def step():
        for _, sl, sb, dl, db in pairs:
            A.remap(ctx, sl, sb, dl, db)

    tuning = {}
    if args.load_tune:
        A.tune_load(ctx, args.load_tune)
        tuning["loaded"] = args.load_tune
    elif not args.no_tune:
        # the autotuner picks each pair's tile shape on these buffers (untimed)
        for name, sl, sb, dl, db in pairs:
            r = A.tune_remap(ctx, sl, sb, dl, db, reps=3)
            tuning[name] = {"shape": r["shape"], "tuned_us": round(r["best_us"], 1),
                            "default_us": round(r["default_us"], 1)}
        log("tuned:", tuning)
        if args.save_tune:
            A.tune_save(ctx, args.save_tune)
    if args.copy_calibration:
        # a plain 1 GiB device copy: its FETCH_SIZE / WRITE_SIZE counters give
        # the scale between counter units and bytes
        log("copy calibration: 1 GiB")
        b[: 1 << 30].copy_(a[: 1 << 30])
        torch.cuda.synchronize()
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    ctx.check()
    # per-launch timing of the dominant kernel with HIP events on its stream
    per = {}
    for name, sl, sb, dl, db in pairs:
        ms, _ = timer.time(lambda: A.remap(ctx, sl, sb, dl, db), reps=10, warm=1)
        per[name] = {"ms": round(ms, 4), "GBps": round(2 * n * 64 / ms / 1e6, 1),
                     "frac": round(2 * n * 64 / ms / 1e6 / HBM_PEAK_GBS, 4)}
    log("per remap:", per)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    ctx.check()
    ms_step = dt / args.steps * 1e3
    value = step_bytes / (dt / args.steps) / 1e9
    avg_ms = float(np.mean([p["ms"] for p in per.values()]))
    achieved = 2 * n * 64 / (avg_ms * 1e-3) / 1e9
    line = {
        "metric": "remap+section GB/s (% HBM peak); program time ADHA vs all-AoS/all-SoA",
        "value": round(value, 1), "unit": "GB/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(ms_step, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "u32", "data": "synthetic",
        "config": {"workload": "single remap: N=2^%d records of 16 x 4-byte fields (8 f32, 8 i32); "
                               "AoS->SoA, SoA->AoS, AoS->AoSoA {0-3},{4-7},{8-15} x64 per step" % args.log2n,
                   "records": n, "record_bytes": 64, "bytes_per_step": step_bytes},
        "frac_of_peak": round(value / HBM_PEAK_GBS, 4),
        "remaps": per,
        "tuning": tuning,
        "shapes": {name: A.get_shape(ctx, sl, dl) for name, sl, _, dl, _ in pairs},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": remap_traffic_bytes() if args.log2n == 26 else None, "traffic_unit": "B per launch",
                     "kernel": "remap_tiles_kernel (persistent LDS-transposing remap)",
                     "per_launch_bytes": 2 * n * 64},
    }
    if not args.only_remap:
        del a, s, t, b
        torch.cuda.empty_cache()
        if not args.skip_probes:
            # the ceilings the fractions are read against, in the same run
            try:
                log("probes")
                line["probes"] = pr = probes_bench(A, synth, torch)
                rf = line["roofline"]
                rf["copy_ceiling"] = pr["copy_GBps"]
                rf["frac_of_copy_ceiling"] = round(rf["achieved"] / pr["copy_GBps"], 4)
                CEIL["copy_GBps"] = pr["copy_GBps"]
                CEIL["read_GBps"] = pr["read_GBps"]
                # random single loads of up to 16 bytes: one 128-byte line each
                rate = max(r["G_accesses_per_s"] for r in pr["random_access"]["rows"] if r["load_bytes"] <= 16)
                CEIL["random_lines_GBps"] = round(rate * 128, 1)
                pr["random_lines_GBps"] = CEIL["random_lines_GBps"]
            except Exception as e:
                line["probes"] = {"error": repr(e)}
            torch.cuda.empty_cache()
        if not args.skip_cpu:
            log("cpu baseline")
            line["cpu_baseline"] = cpu_baseline(synth)
        if not args.skip_program:
            try:
                line["program"] = program_bench(A, synth, torch, timer, args.program_log2n, cap_bytes=args.cap_bytes)
            except Exception as e:  # report, keep the main line
                line["program"] = {"error": repr(e)}
            torch.cuda.empty_cache()
        if not args.skip_kmeans:
            try:
                line["kmeans"] = kmeans_bench(A, synth, torch, timer)
            except Exception as e:
                line["kmeans"] = {"error": repr(e)}
            torch.cuda.empty_cache()
        if not args.skip_medical:
            try:
                line["medical"] = medical_bench(A, synth, torch, timer)
            except Exception as e:
                line["medical"] = {"error": repr(e)}
            torch.cuda.empty_cache()
        if not args.skip_medical_narrow:
            try:
                line["medical_narrow"] = medical_bench(A, synth, torch, timer, narrow=True)
            except Exception as e:
                line["medical_narrow"] = {"error": repr(e)}
            torch.cuda.empty_cache()
        if not args.skip_flow:
            try:
                line["flow"] = flow_bench(A, synth, torch, timer, args.program_log2n)
            except Exception as e:
                line["flow"] = {"error": repr(e)}
            torch.cuda.empty_cache()
        if not args.skip_hetero:
            try:
                line["hetero"] = hetero_bench(A, synth, torch)
            except Exception as e:
                line["hetero"] = {"error": repr(e)}
            torch.cuda.empty_cache()
        if not args.skip_subdword:
            try:
                line["subdword"] = subdword_bench(A, torch, timer)
            except Exception as e:
                line["subdword"] = {"error": repr(e)}
            torch.cuda.empty_cache()
        if not args.skip_batched:
            try:
                line["batched"] = batched_bench(A, synth, torch, timer)
            except Exception as e:
                line["batched"] = {"error": repr(e)}
            torch.cuda.empty_cache()
        if not args.skip_learned:
            try:
                line["learned"] = learned_bench(A, synth, torch, args)
            except Exception as e:
                line["learned"] = {"error": repr(e)}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
