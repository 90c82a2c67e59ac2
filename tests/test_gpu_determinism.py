"""Determinism: repeated calls on the same input give the same bytes.

- argsort (stable, so its output is unique) ten times in a row;
- one bucketing level with a fixed node seed (samples, model b and T, bucket
  sizes and, with a payload, the stable partition) five times;
- a segmented batch with a payload replayed from its captured graph five
  times, with the program's own eager work between the replays."""
import numpy as np
import pytest

from paper_2405_07122_amd import datagen
from tests.gpu_util import banner, to_dev, to_host

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2405_07122_amd import pcfsort
    pcfsort.load()
    return pcfsort


def test_argsort_repeats_bit_identical(P):
    import torch
    n = 3_000_017
    banner(f"determinism: argsort x10, n={n}")
    d = to_dev(datagen.f64("mix8", n, 21))
    ws = P.workspace(P.KEY_F64, n, True)
    k0, i0 = P.pcf_argsort(d, ws=ws)
    ko = torch.empty_like(k0)
    io = torch.empty_like(i0)
    for _ in range(9):
        P.pcf_argsort(d, keys_out=ko, idx_out=io, ws=ws)
        assert torch.equal(ko, k0) and torch.equal(io, i0)
    ref_v, ref_i = torch.sort(d, stable=True)
    assert torch.equal(k0, ref_v) and torch.equal(i0.long(), ref_i)


def test_level_trace_repeats_bit_identical(P):
    import torch
    n = 2_000_000
    banner(f"determinism: level trace x5, n={n}")
    d = to_dev(datagen.f64("lognormal", n, 22))
    v = torch.arange(n, dtype=torch.int32, device="cuda")
    first = P.pcf_level_trace(d, 4096, 4095, 255, 0xabcdef, vals=v)
    for _ in range(4):
        t = P.pcf_level_trace(d, 4096, 4095, 255, 0xabcdef, vals=v)
        for k in ("b", "T", "sizes"):
            np.testing.assert_array_equal(t[k], first[k])
        assert torch.equal(t["part_keys"], first["part_keys"])
        assert torch.equal(t["part_vals"], first["part_vals"])


def test_segmented_graph_replays_bit_identical(P):
    import torch
    banner("determinism: segmented graph replays x5")
    keys, offsets, vals = datagen.segments(num=96, lo_log2=8, hi_log2=18, seed=23)
    n = int(offsets[-1])
    dk, dv = to_dev(keys), to_dev(vals)
    doff = to_dev(offsets.view(np.int64))
    ws = P.workspace(P.KEY_F64, n, True, 96)
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    k0, v0 = P.pcf_sort_segmented(dk, doff, dv, ws=ws, d_status=st)
    torch.cuda.synchronize()
    assert int(st.cpu()[0]) == 0
    ko, vo = torch.empty_like(k0), torch.empty_like(v0)
    for _ in range(5):
        ko.zero_()
        vo.zero_()
        P.pcf_sort_segmented(dk, doff, dv, keys_out=ko, vals_out=vo, ws=ws, d_status=st)
        P.pcf_sort_f64(torch.randn(1 << 15, dtype=torch.float64, device="cuda"))  # eager work between
        torch.cuda.synchronize()
        assert int(st.cpu()[0]) == 0
        assert torch.equal(ko, k0) and torch.equal(vo, v0)
    for s in range(0, 96, 7):
        a, b = int(offsets[s]), int(offsets[s + 1])
        order = np.argsort(keys[a:b], kind="stable")
        np.testing.assert_array_equal(to_host(k0, np.float64)[a:b], keys[a:b][order])
        np.testing.assert_array_equal(to_host(v0, np.uint32)[a:b], vals[a:b][order])
    P.pcf_graph_clear()
