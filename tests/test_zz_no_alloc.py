"""The allocation-free entry point adha_section_run_static against
adha_section_run: a reduction's partials come from the library's static
device array instead of the context's own allocation; the kernels and the
order of every sum are the same, so the tables must match bit for bit (and
the oracle within 1 ulp).  Two calls in a row, the second on a smaller
input, and then the other kernel forms."""
import numpy as np
import pytest
import torch

import oracle
from oracle import reduce as OR
from oracle.layout import aos as oaos, soa as osoa
from paper_1407_4859_amd import adha as A
from paper_1407_4859_amd import synth
from gpu_util import dev_bytes, host, mirror, say
from test_gpu_reduce import _check, _struct, _wide_struct

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    return A.Ctx(0)


def _both(ctx, spec, cols, O, read, key, n_keys):
    st = A.Struct.from_spec(spec)
    L = mirror(st, O)
    buf_h = oracle.pack(O, cols)
    dev = dev_bytes(buf_h)
    cells = n_keys * (len(read) + 1)
    out = torch.full((cells * 8,), 0xEE, dtype=torch.uint8, device="cuda")
    sec = A.Section.reduce(st, read, key, n_keys, out)
    say("no-alloc: static entry", spec.n, "records", n_keys, "keys")
    A.section_run_static(ctx, sec, L, dev)
    ctx.check()
    got_static = host(out).copy()
    out.fill_(0x11)
    A.section_run(ctx, sec, L, dev)
    ctx.check()
    got = host(out).copy()
    table, bad = OR.reduce(O, spec.dtypes, read, key, n_keys, buf_h)
    assert bad == 0
    return got_static, got, table


def test_static_reduction_matches_allocating_entry_twice(ctx):
    # first call: 2^18 + 5 records, 5 keys (register form)
    n1 = (1 << 18) + 5
    spec, cols = _wide_struct(n1, 21, 5, True)
    read = [0, 1, 2, 4, 5, 6]
    a_static, a, table = _both(ctx, spec, cols, osoa(n1, spec.elem_bytes), read, 3, 5)
    assert np.array_equal(a_static, a)
    _check(a_static.view(np.uint64), table, spec.dtypes, read)
    # second call, right after, on a smaller input
    n2 = 1003
    spec2, cols2 = _wide_struct(n2, 22, 5, False)
    b_static, b, table2 = _both(ctx, spec2, cols2, oaos(n2, spec2.elem_bytes), read, 3, 5)
    assert np.array_equal(b_static, b)
    _check(b_static.view(np.uint64), table2, spec2.dtypes, read)


@pytest.mark.parametrize("n_keys,n", [(64, 50_000), (409, 7_001), (1, 1 << 16)])
def test_static_reduction_other_forms(ctx, n_keys, n):
    spec, cols = _struct(n, 23, n_keys)
    read = [0, 2, 5, 7, 8, 10] if n_keys < 409 else [0, 7, 8]
    key = -1 if n_keys == 1 else 6
    s, a, table = _both(ctx, spec, cols, osoa(n, spec.elem_bytes), read, key, n_keys)
    assert np.array_equal(s, a)
    _check(s.view(np.uint64), table, spec.dtypes, read)


def test_static_entry_runs_other_sections_unchanged(ctx):
    n = 70_001
    spec = synth.config3_struct(n)
    st = A.Struct.from_spec(spec)
    cols = synth.record_matrix(3, n, spec.dtypes, spec.elem_bytes)
    O = osoa(n, spec.elem_bytes)
    L = mirror(st, O)
    buf_h = oracle.pack(O, cols)
    idx = synth.uniform_index_torch(3, 5, n * 16, n, "cuda")
    for s in synth.random_program(3, spec.n_fields)[:4]:
        sec = A.Section.from_spec(st, s)
        d1, d2 = dev_bytes(buf_h), dev_bytes(buf_h)
        A.section_run_static(ctx, sec, L, d1, idx if s.degree else None)
        A.section_run(ctx, sec, L, d2, idx if s.degree else None)
        ctx.check()
        assert torch.equal(d1, d2), s
