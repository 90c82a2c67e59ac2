"""GPU checks at the benchmark's full sizes, in the benchmark's launch
configuration (default policy, caller workspace).

At n = 1e8 the output is compared element by element with the CPU oracle for
the uniform array, and with torch's sort (a library sort on the same device,
independent of this library) for every distribution; argsort indices of
every distribution with torch's stable sort.  The uint64 kinds run at 2e8
keys.  The batched workload (2048 segments, about 1.09e9 keys with a uint32
payload) is compared per segment with torch's stable sorts (by key, then by
segment).  A 5e8-key array generated on the device checks the largest size."""
import numpy as np
import pytest

from paper_2405_07122_amd import datagen
from tests.gpu_util import banner, to_dev, to_host

pytestmark = pytest.mark.gpu

N = 100_000_000


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2405_07122_amd import pcfsort
    pcfsort.load()
    return pcfsort


@pytest.fixture(scope="module")
def ws(P):
    return P.workspace(P.KEY_F64, N, with_payload=True)


@pytest.mark.parametrize("dist", datagen.F64_DISTS)
def test_fullsize_f64_vs_library_sort(P, ws, dist):
    import torch
    banner(f"full size {dist} n={N}")
    x = to_dev(datagen.config2(dist, N))
    out = P.pcf_sort_f64(x, ws=ws)
    ref, _ = torch.sort(x)
    assert torch.equal(out, ref)


def test_fullsize_uniform_vs_oracle(P, ws, oracle):
    banner("full size uniform vs oracle")
    xh = datagen.config2("uniform", N)
    ref, _, _ = oracle.sort(xh)
    got = to_host(P.pcf_sort_f64(to_dev(xh), ws=ws), np.float64)
    np.testing.assert_array_equal(got, ref)


@pytest.mark.parametrize("dist", datagen.F64_DISTS)
def test_fullsize_argsort(P, ws, dist):
    import torch
    banner(f"full size argsort {dist}")
    x = to_dev(datagen.config2(dist, N))
    k, idx = P.pcf_argsort(x, ws=ws)
    rk, ri = torch.sort(x, stable=True)
    assert torch.equal(k, rk)
    assert torch.equal(idx.to(torch.int64), ri)


@pytest.mark.parametrize("kind,n", [("clustered", 200_000_000), ("bursty", 200_000_000),
                                    ("zipf", 200_000_000)])
def test_fullsize_u64(P, kind, n):
    import torch
    banner(f"full size u64 {kind} n={n}")
    xh = datagen.u64(kind, n, datagen.U64_SEEDS[kind])
    x = to_dev(xh)
    out = P.pcf_sort_u64(x)
    # order of unsigned values: compare on the host for a sample, and check
    # sortedness + multiset on the device through the signed view
    flip = torch.tensor(-(2**63), dtype=torch.int64, device="cuda")
    ref, _ = torch.sort(x ^ flip)
    assert torch.equal(out ^ flip, ref)


@pytest.mark.parametrize("payload", [True, False])
def test_fullsize_batched_segments(P, ws, payload):
    """The batched workload exactly as the benchmark runs it (graph path, caller
    workspace), with its payload and keys alone (the keys-only scatter over
    nodes of very uneven sizes), against an independent segmented stable sort
    built from two stable torch sorts: by key, then by segment."""
    import torch
    keys, offsets, vals = datagen.segments(num=2048)
    n = int(offsets[-1])
    banner(f"full size batched: 2048 segments, {n} keys, payload={payload}")
    dk = to_dev(keys)
    dv = to_dev(vals) if payload else None
    doff = to_dev(offsets.view(np.int64))
    del keys, vals
    wsb = P.workspace(P.KEY_F64, n, payload, 2048)
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    ko, vo = P.pcf_sort_segmented(dk, doff, dv, ws=wsb, d_status=st)
    torch.cuda.synchronize()
    assert int(st.cpu()[0]) == 0
    del wsb
    _, p1 = torch.sort(dk, stable=True)
    seg = torch.searchsorted(doff, torch.arange(n, device="cuda", dtype=torch.int64),
                             right=True) - 1
    _, p2 = torch.sort(seg[p1], stable=True)
    del seg
    perm = p1[p2]
    del p1, p2
    assert torch.equal(ko, dk[perm])
    if payload:
        assert torch.equal(vo, dv[perm])
    P.pcf_graph_clear()


def test_largest_size_device_generated(P):
    import torch
    n = 500_000_000
    banner(f"largest size n={n}")
    g = torch.Generator(device="cuda").manual_seed(7)
    x = torch.rand(n, dtype=torch.float64, device="cuda", generator=g)
    out = P.pcf_sort_f64(x)
    assert bool((out[1:] >= out[:-1]).all())
    ref, _ = torch.sort(x)
    assert torch.equal(out, ref)
