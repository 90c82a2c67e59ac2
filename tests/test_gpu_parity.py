"""GPU parity: the HIP library against the CPU oracle, bit for bit.

Every comparison is exact: the sorted order of keys without NaN / -0.0 is
unique, argsort ties break by position, and one bucketing level with the same
parameters and node seed must reproduce the oracle's model (b, T), bucket sizes
and stable partition exactly (both sides round the fp64 bin function the same
way)."""
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


def _dt(x):
    return np.float64 if x.dtype == np.float64 else np.uint64


def _halved_range_keys():
    """Keys whose range width x_max - x_min overflows fp64 (about +-1.7e308): a
    grid k 2^1020 (k = -8..8) plus keys spread over the whole range."""
    rng = np.random.default_rng(36)
    grid = np.arange(-8, 9, dtype=np.float64) * 2.0 ** 1020
    x = np.concatenate([np.tile(grid, 600), rng.uniform(-1.0, 1.0, 40_000) * 1.7e308])
    return x[rng.permutation(x.shape[0])] + 0.0


LEVEL_CASES = [
    ("uniform", lambda: datagen.f64("uniform", 200_000, 31), (4096, 8192, 511)),
    ("lognormal", lambda: datagen.f64("lognormal", 150_000, 32), (2000, 16000, 1023)),
    ("normal-ragged", lambda: datagen.f64("normal", 99_991, 33), (777, 3001, 300)),
    ("zipf-u64", lambda: datagen.u64("zipf", 120_000, 34, distinct=5000), (3000, 5000, 255)),
    ("bursty-u64", lambda: datagen.u64("bursty", 100_003, 35), (1500, 4000, 2047)),
    ("two-valued", lambda: np.where(np.random.default_rng(3).random(50_000) < 0.4, 1.5, -2.25),
     (500, 700, 63)),
    ("halved-range", _halved_range_keys, (2000, 4096, 255)),
]


@pytest.mark.parametrize("name,gen,params", LEVEL_CASES, ids=[c[0] for c in LEVEL_CASES])
def test_level_trace_matches_oracle(P, oracle, name, gen, params):
    x = gen()
    alpha, beta, gamma = params
    banner(f"level trace {name} n={x.shape[0]} alpha={alpha} beta={beta} gamma={gamma}")
    nseed = oracle.node_seed(7, 0, 0, 0)
    idx = np.arange(x.shape[0], dtype=np.uint32)
    ref = oracle.level(x, alpha, beta, gamma, nseed, vals=idx)
    got = P.pcf_level_trace(to_dev(x), alpha, beta, gamma, nseed, vals=to_dev(idx))
    assert got["status"] == ref.status
    assert got["min_bits"] == ref.min_bits and got["max_bits"] == ref.max_bits
    assert got["scale_bits"] == np.float64(ref.scale).view(np.uint64)
    assert got["halves"] == ref.halves
    np.testing.assert_array_equal(got["b"], ref.b)
    np.testing.assert_array_equal(got["T"], ref.T)
    np.testing.assert_array_equal(got["sizes"], ref.sizes)
    np.testing.assert_array_equal(to_host(got["part_keys"], _dt(x)), ref.part_keys)
    np.testing.assert_array_equal(to_host(got["part_vals"], np.uint32), ref.part_vals)


SIZES = [1, 2, 3, 99, 100, 101, 2047, 2048, 2049, 8191, 8192, 8193, 12_345, 65_537, 300_001]


@pytest.mark.parametrize("n", SIZES)
def test_sort_sizes_f64(P, oracle, n):
    banner(f"sort f64 uniform n={n}")
    x = datagen.f64("normal", n, 1000 + n)
    ref, _, _ = oracle.sort(x)
    got = to_host(P.pcf_sort_f64(to_dev(x)), np.float64)
    np.testing.assert_array_equal(got, ref)


def test_config1_bit_exact(P, oracle):
    banner("config1: n=1e6 fp64 uniform seed 0")
    x = datagen.config1()
    ref, _, _ = oracle.sort(x)
    got = to_host(P.pcf_sort_f64(to_dev(x)), np.float64)
    np.testing.assert_array_equal(got, ref)
    np.testing.assert_array_equal(got, np.sort(x))


@pytest.mark.parametrize("dist", datagen.F64_DISTS)
def test_argsort_f64(P, oracle, dist):
    n = 400_000
    banner(f"argsort f64 {dist} n={n}")
    x = datagen.f64(dist, n, 77)
    x = np.round(x, 3) + 0.0  # duplicates, so ties matter
    ks, idx, _ = oracle.argsort(x)
    gk, gi = P.pcf_argsort(to_dev(x))
    np.testing.assert_array_equal(to_host(gk, np.float64), ks)
    np.testing.assert_array_equal(to_host(gi, np.uint32), idx)


@pytest.mark.parametrize("kind", datagen.U64_KINDS)
def test_sort_u64(P, oracle, kind):
    n = 500_000
    banner(f"sort u64 {kind} n={n}")
    x = datagen.u64(kind, n, 88, distinct=20_000)
    ref, _, _ = oracle.sort(x)
    got = to_host(P.pcf_sort_u64(to_dev(x)), np.uint64)
    np.testing.assert_array_equal(got, ref)
    ks, idx, _ = oracle.argsort(x)
    gk, gi = P.pcf_argsort(to_dev(x))
    np.testing.assert_array_equal(to_host(gi, np.uint32), idx)


def test_invalid_keys(P):
    for bad in (np.nan, np.inf, -np.inf, -0.0):
        for n in (50, 5000, 100_000):
            banner(f"invalid key {bad} n={n}")
            x = datagen.f64("uniform", n, 5)
            x[n // 2] = bad
            with pytest.raises(P.PcfError) as e:
                P.pcf_sort_f64(to_dev(x))
            assert e.value.code == P.ERR_INVALID_KEY


def test_in_place_and_all_equal(P, oracle):
    import torch
    banner("in place + all equal")
    x = datagen.f64("exponential", 250_000, 9)
    t = to_dev(x)
    P.pcf_sort_f64(t, out=t)
    np.testing.assert_array_equal(to_host(t, np.float64), np.sort(x))
    y = np.full(300_000, 3.5)
    _, gi = P.pcf_argsort(to_dev(y))
    np.testing.assert_array_equal(to_host(gi, np.uint32), np.arange(300_000, dtype=np.uint32))


def test_level_trace_keys_only_multiset(P, oracle):
    """Keys alone are scattered with unstable ranks (equal keys are the same
    bits): the model and the sizes are exact, each bucket is the oracle's as
    a multiset."""
    import torch
    x = datagen.f64("normal", 250_000, 41)
    alpha, beta, gamma = 4096, 4095, 255
    nseed = oracle.node_seed(9, 0, 0, 0)
    banner("level trace keys only")
    ref = oracle.level(x, alpha, beta, gamma, nseed)
    got = P.pcf_level_trace(to_dev(x), alpha, beta, gamma, nseed)
    np.testing.assert_array_equal(got["b"], ref.b)
    np.testing.assert_array_equal(got["T"], ref.T)
    np.testing.assert_array_equal(got["sizes"], ref.sizes)
    part = to_host(got["part_keys"], np.float64)
    bounds = np.concatenate([[0], np.cumsum(ref.sizes.astype(np.int64))])
    for j in range(gamma + 1):
        a, b = bounds[j], bounds[j + 1]
        np.testing.assert_array_equal(np.sort(part[a:b]), np.sort(ref.part_keys[a:b]))


SEG_SIZES = [0, 1, 5, 99, 100, 101, 2047, 2048, 2049, 4096, 4097, 8192, 8193, 0, 20_000,
             150_000, 3, 70_001]


def _segments(kind):
    rng = np.random.default_rng(5)
    parts = []
    for i, m in enumerate(SEG_SIZES):
        if kind == "f64":
            parts.append(datagen.f64(datagen.F64_DISTS[i % 6], m, 300 + i))
        else:
            parts.append(datagen.u64(datagen.U64_KINDS[i % 3], m, 400 + i, distinct=5000)
                         if m else np.zeros(0, np.uint64))
    keys = np.concatenate(parts)
    offsets = np.zeros(len(SEG_SIZES) + 1, dtype=np.uint64)
    offsets[1:] = np.cumsum(SEG_SIZES)
    vals = np.concatenate([rng.integers(0, 2**32, m, dtype=np.uint64).astype(np.uint32)
                           for m in SEG_SIZES])
    return keys, offsets, vals


@pytest.mark.parametrize("kind", ["f64", "u64"])
@pytest.mark.parametrize("payload", [False, True])
def test_segmented_matches_oracle(P, oracle, kind, payload):
    banner(f"segmented {kind} payload={payload}")
    keys, offsets, vals = _segments(kind)
    ref_k, ref_v = oracle.sort_segmented(keys, offsets, vals if payload else None)
    dt = np.float64 if kind == "f64" else np.uint64
    gk, gv = P.pcf_sort_segmented(to_dev(keys), to_dev(offsets.view(np.int64)),
                                  to_dev(vals) if payload else None)
    np.testing.assert_array_equal(to_host(gk, dt), ref_k)
    if payload:
        np.testing.assert_array_equal(to_host(gv, np.uint32), ref_v)


def test_segmented_equals_per_array_plain(P):
    """Batching changes nothing: each segment equals the plain sort of it."""
    banner("segmented vs plain per segment")
    keys, offsets, vals = datagen.segments(num=64, lo_log2=6, hi_log2=17, seed=12)
    gk, gv = P.pcf_sort_segmented(to_dev(keys), to_dev(offsets.view(np.int64)), to_dev(vals))
    gk = to_host(gk, np.float64)
    gv = to_host(gv, np.uint32)
    for s in range(64):
        a, b = int(offsets[s]), int(offsets[s + 1])
        if b == a:
            continue
        pk, pi = P.pcf_argsort(to_dev(keys[a:b]))
        np.testing.assert_array_equal(gk[a:b], to_host(pk, np.float64))
        # the payload is the in-segment index, so it equals the argsort
        np.testing.assert_array_equal(gv[a:b], to_host(pi, np.uint32))


def _segment_data(kind, seed):
    """Same segment sizes as _segments, new contents per seed."""
    rng = np.random.default_rng(seed)
    parts = []
    for i, m in enumerate(SEG_SIZES):
        if kind == "f64":
            parts.append(datagen.f64(datagen.F64_DISTS[(i + seed) % 6], m, seed * 100 + i))
        else:
            parts.append(datagen.u64(datagen.U64_KINDS[(i + seed) % 3], m, seed * 100 + i,
                                     distinct=5000) if m else np.zeros(0, np.uint64))
    vals = rng.integers(0, 2**32, sum(SEG_SIZES), dtype=np.uint64).astype(np.uint32)
    return np.concatenate(parts), vals


@pytest.mark.parametrize("kind", ["f64", "u64"])
@pytest.mark.parametrize("payload", [False, True])
def test_segmented_graph_replays(P, oracle, kind, payload):
    """With a caller workspace the segmented call is captured once and replayed;
    every replay reads the buffers' current contents and matches the oracle,
    with unrelated eager work between replays, and a data error in one replay
    does not leak into the next."""
    import torch
    banner(f"segmented graph replays {kind} payload={payload}")
    dt = np.float64 if kind == "f64" else np.uint64
    tdt = torch.float64 if kind == "f64" else torch.int64
    offsets = np.zeros(len(SEG_SIZES) + 1, dtype=np.uint64)
    offsets[1:] = np.cumsum(SEG_SIZES)
    n = int(offsets[-1])
    d_keys = torch.empty(n, dtype=tdt, device="cuda")
    d_vals = torch.empty(n, dtype=torch.int32, device="cuda") if payload else None
    d_off = to_dev(offsets.view(np.int64))
    k_out = torch.empty_like(d_keys)
    v_out = torch.empty_like(d_vals) if payload else None
    ws = P.workspace(P.KEY_F64 if kind == "f64" else P.KEY_U64, n, payload, len(SEG_SIZES))
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    s0 = P.pcf_graph_stats()
    for rep in range(5):
        keys, vals = _segment_data(kind, 20 + rep)
        bad = rep == 2 and kind == "f64"
        if bad:
            keys = keys.copy()
            keys[int(offsets[5]) + 3] = np.nan
        d_keys.copy_(to_dev(keys))
        if payload:
            d_vals.copy_(to_dev(vals))
        P.pcf_sort_segmented(d_keys, d_off, d_vals, keys_out=k_out, vals_out=v_out, ws=ws,
                             d_status=st)
        # unrelated eager work on the same stream between replays
        junk = torch.randn(1 << 16, device="cuda", dtype=torch.float64)
        P.pcf_sort_f64(junk)
        torch.cuda.synchronize()
        code = int(st.cpu()[0])
        if bad:
            assert code == P.ERR_INVALID_KEY
            continue
        assert code == 0
        ref_k, ref_v = oracle.sort_segmented(keys, offsets, vals if payload else None)
        np.testing.assert_array_equal(to_host(k_out, dt), ref_k)
        if payload:
            np.testing.assert_array_equal(to_host(v_out, np.uint32), ref_v)
    s1 = P.pcf_graph_stats()
    assert s1["captures"] - s0["captures"] == 1
    assert s1["replays"] - s0["replays"] == 4


def test_segmented_graph_in_place_and_no_status(P, oracle):
    """In-place replays (keys_in == keys_out) and the synchronous form without a
    status word, which reports an invalid key through its return code."""
    import torch
    banner("segmented graph in place")
    offsets = np.zeros(len(SEG_SIZES) + 1, dtype=np.uint64)
    offsets[1:] = np.cumsum(SEG_SIZES)
    n = int(offsets[-1])
    d = torch.empty(n, dtype=torch.float64, device="cuda")
    d_off = to_dev(offsets.view(np.int64))
    ws = P.workspace(P.KEY_F64, n, False, len(SEG_SIZES))
    for rep in range(3):
        keys, _ = _segment_data("f64", 40 + rep)
        d.copy_(to_dev(keys))
        P.pcf_sort_segmented(d, d_off, None, keys_out=d, ws=ws)
        ref_k, _ = oracle.sort_segmented(keys, offsets, None)
        np.testing.assert_array_equal(to_host(d, np.float64), ref_k)
    keys[17] = np.inf
    d.copy_(to_dev(keys))
    with pytest.raises(P.PcfError) as ei:
        P.pcf_sort_segmented(d, d_off, None, keys_out=d, ws=ws)
    assert ei.value.code == P.ERR_INVALID_KEY
    P.pcf_graph_clear()
    assert P.pcf_graph_stats()["cached"] == 0
