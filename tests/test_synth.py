"""The shared input generator: published SplitMix64 values, and the numpy,
scalar and torch forms agree (CPU only)."""
import numpy as np
import torch

from paper_1407_4859_amd import synth


def test_published_splitmix64_sequence():
    # SplitMix64 started from state 0 (seed 0, stream 0) yields these first outputs
    want = [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]
    assert [synth.splitmix64_scalar(0, 0, i) for i in range(3)] == want
    assert [int(v) for v in synth.splitmix64(0, 0, 0, 3)] == want


def test_forms_agree():
    for seed, stream, start in ((1, 0, 0), (3, 31, 1000), (255, (1 << 20) - 1, 12345)):
        a = synth.splitmix64(seed, stream, start, 4096)
        t = synth.splitmix64_torch(seed, stream, start, 4096, "cpu").numpy().view(np.uint64)
        assert np.array_equal(a, t)
        assert int(a[17]) == synth.splitmix64_scalar(seed, stream, start + 17)
        for dt, e in ((synth.F32, 4), (synth.F64, 8), (synth.I32, 4), (synth.RAW, 4),
                      (synth.RAW, 8), (synth.RAW, 2), (synth.RAW, 1)):
            d = synth.decode(a, dt, e)
            dtt = synth.decode_torch(torch.from_numpy(a.view(np.int64)), dt, e).numpy()
            assert np.array_equal(d, dtt)


def test_draws_at_counters_match_the_sequence():
    rng = np.random.default_rng(0)
    recs = rng.integers(0, 1 << 24, 300)
    full = synth.splitmix64(3, 7, 0, 1 << 24)
    assert np.array_equal(synth.splitmix64_at(3, 7, recs), full[recs])
    for dt, e in ((synth.F32, 4), (synth.F64, 8), (synth.I32, 4)):
        assert np.array_equal(synth.field_values_at(3, 7, recs, dt, e), synth.decode(full[recs], dt, e))
    ix = synth.uniform_index(3, 999, 1 << 20, 12345)
    c = rng.integers(0, 1 << 20, 500)
    assert np.array_equal(synth.uniform_index_at(3, 999, c, 12345), ix[c])


def test_value_ranges():
    f = synth.field_values(2, 0, 100000, synth.F32).view(np.float32)
    assert f.min() >= -1.0 and f.max() < 1.0
    d = synth.field_values(2, 1, 100000, synth.F64, 8).view(np.float64)
    assert d.min() >= -1.0 and d.max() < 1.0
    i = synth.field_values(2, 2, 100000, synth.I32).view(np.int32)
    assert i.min() >= 0
    ix = synth.uniform_index(2, 3, 100000, 77)
    assert ix.min() == 0 and ix.max() == 76
    ixt = synth.uniform_index_torch(2, 3, 100000, 77, "cpu").numpy()
    assert np.array_equal(ix, ixt)


def test_workload_shapes():
    st = synth.config3_struct()
    assert st.n == 1 << 24 and st.record_bytes == 144 and st.n_fields == 32
    secs = synth.random_program(3, 32)
    assert len(secs) == 8 and sum(s.degree == 16 for s in secs) == 4
    for s in secs:
        assert 2 <= len(s.read) <= 10 and 1 <= len(s.write) <= 2
        assert not set(s.read) & set(s.write)
    arrs = synth.config4_arrays()
    assert len(arrs) == 512
    for a in arrs:
        assert 1 << 10 <= a["n"] < 1 << 22 and 4 <= len(a["elem_bytes"]) <= 24
        assert set(a["elem_bytes"]) <= {4, 8}
    assert synth.config2_struct().record_bytes == 64
