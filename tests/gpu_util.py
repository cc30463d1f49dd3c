"""Helpers shared by the GPU tests: device buffers from oracle-packed host
images, and comparison of device results with oracle results."""
import sys

import numpy as np
import torch

from oracle.layout import Layout as OLayout
from paper_1407_4859_amd import adha as A
from paper_1407_4859_amd import synth


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def dev_bytes(host: np.ndarray, extra: int = 0, fill: int = 0xA5):
    """uint8 device tensor holding `host` (plus `extra` bytes of `fill`)."""
    t = torch.full((max(1, host.size + extra),), fill, dtype=torch.uint8, device="cuda")
    if host.size:
        t[: host.size].copy_(torch.from_numpy(host))
    return t


def dev_empty(n: int, fill: int = 0xA5):
    return torch.full((max(1, n),), fill, dtype=torch.uint8, device="cuda")


def host(t, n=None):
    a = t.cpu().numpy()
    return a if n is None else a[:n]


def mirror(st: A.Struct, O: OLayout) -> A.Layout:
    """The library layout with the oracle layout's partition and tiles."""
    gof = [O.group_of[f] for f in range(len(O.elem_bytes))]
    tiles = [t for _, t in O.groups]
    return A.Layout.create(st, gof, tiles)


def first_diff(a: np.ndarray, b: np.ndarray):
    d = np.nonzero(a != b)[0]
    return None if d.size == 0 else (int(d[0]), int(a[d[0]]), int(b[d[0]]), int(d.size))


def fill_aos_device(spec, seed: int, extra: int = 0):
    """Device buffer holding the seeded values of every record packed in field
    order (field f of record r at r * S + sum of the earlier element sizes),
    drawn on the device by the torch form of the generator."""
    n, S = spec.n, spec.record_bytes
    t = torch.zeros(max(1, n * S + extra), dtype=torch.uint8, device="cuda")
    view = t[: n * S].view(n, S)
    chunk = 1 << 24
    off = 0
    for f, (dt, e) in enumerate(zip(spec.dtypes, spec.elem_bytes)):
        for s in range(0, n, chunk):
            c = min(chunk, n - s)
            z = synth.splitmix64_torch(seed, f, s, c, "cuda")
            view[s:s + c, off:off + e] = synth.decode_torch(z, dt, e)
        off += e
    return t


def host_cores(cap: int = 16) -> int:
    """Host threads the oracle may use (the CPU share given to this process)."""
    import os
    try:
        return max(1, min(cap, len(os.sched_getaffinity(0))))
    except AttributeError:
        return 1


def oracle_remap_threaded(src_layout: OLayout, src: np.ndarray, dst_layout: OLayout,
                          threads: int = 0) -> np.ndarray:
    """The oracle's remap of a whole buffer, its record range split over host
    threads (records are independent; every thread writes its own records
    into the one zero-filled destination)."""
    from concurrent.futures import ThreadPoolExecutor
    import oracle
    n = src_layout.n
    t = threads or host_cores()
    out = np.zeros(dst_layout.nbytes, np.uint8)
    bounds = [n * i // t for i in range(t + 1)]
    with ThreadPoolExecutor(t) as ex:
        list(ex.map(lambda i: oracle.remap(src_layout, src, dst_layout, bounds[i], bounds[i + 1], out=out),
                    range(t)))
    return out
