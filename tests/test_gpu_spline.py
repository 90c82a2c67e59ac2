"""Spline Learned Sort on the GPU (App. A.5; policy model = 1) against the
oracle's spline model: one bucketing level bit for bit (prefix counts, bucket
sizes, stable partition), and whole sorts, argsorts and segmented sorts."""
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
    base = pcfsort.get_policy()
    pcfsort.set_policy(model=1)
    yield pcfsort
    pcfsort.set_policy(**base)


def _dt(x):
    return np.float64 if x.dtype == np.float64 else np.uint64


LEVEL_CASES = [
    ("uniform", lambda: datagen.f64("uniform", 200_000, 41), (4096, 8192, 511)),
    ("lognormal", lambda: datagen.f64("lognormal", 150_000, 42), (2000, 16000, 1023)),
    ("normal-ragged", lambda: datagen.f64("normal", 99_991, 43), (777, 3001, 300)),
    ("zipf-u64", lambda: datagen.u64("zipf", 120_000, 44, distinct=5000), (3000, 5000, 255)),
    ("bursty-u64", lambda: datagen.u64("bursty", 100_003, 45), (1500, 4000, 2047)),
    ("mix8", lambda: datagen.f64("mix8", 80_000, 46), (65535, 9000, 700)),
]


@pytest.mark.parametrize("name,gen,params", LEVEL_CASES, ids=[c[0] for c in LEVEL_CASES])
def test_spline_level_matches_oracle(P, oracle, name, gen, params):
    x = gen()
    alpha, beta, gamma = params
    banner(f"spline level {name} n={x.shape[0]} alpha={alpha} beta={beta} gamma={gamma}")
    nseed = oracle.node_seed(9, 0, 0, 0)
    idx = np.arange(x.shape[0], dtype=np.uint32)
    ref = oracle.level(x, alpha, beta, gamma, nseed, vals=idx, model="spline")
    got = P.pcf_level_trace(to_dev(x), alpha, beta, gamma, nseed, vals=to_dev(idx))
    assert got["status"] == ref.status
    assert got["scale_bits"] == np.float64(ref.scale).view(np.uint64)
    np.testing.assert_array_equal(got["b"], ref.b)
    np.testing.assert_array_equal(got["T"], ref.b)  # the spline's table is b itself
    np.testing.assert_array_equal(got["sizes"], ref.sizes)
    np.testing.assert_array_equal(to_host(got["part_keys"], _dt(x)), ref.part_keys)
    np.testing.assert_array_equal(to_host(got["part_vals"], np.uint32), ref.part_vals)


@pytest.mark.parametrize("dist", ["uniform", "normal", "lognormal", "mix8"])
def test_spline_sort_and_argsort(P, oracle, dist):
    banner(f"spline sort {dist}")
    x = datagen.f64(dist, 400_003, 50)
    ref, ridx, _ = oracle.argsort(x, model="spline")
    d = to_dev(x)
    np.testing.assert_array_equal(to_host(P.sort(d), np.float64), ref)
    k, i = P.pcf_argsort(d)
    np.testing.assert_array_equal(to_host(i, np.uint32), ridx)


@pytest.mark.parametrize("kind", ["zipf", "clustered", "bursty"])
def test_spline_u64(P, oracle, kind):
    banner(f"spline u64 {kind}")
    x = datagen.u64(kind, 300_000, 51, distinct=4000)
    ref, _, _ = oracle.sort(x, model="spline")
    np.testing.assert_array_equal(to_host(P.sort(to_dev(x)), np.uint64), ref)


def test_spline_segmented_and_large(P, oracle):
    import torch
    banner("spline segmented + 4e7")
    keys, offsets, vals = datagen.segments(num=40, lo_log2=6, hi_log2=16, seed=52)
    rk, rv = oracle.sort_segmented(keys, offsets, vals, model="spline")
    ws = P.workspace(P.KEY_F64, keys.shape[0], True, 40)
    gk, gv = P.pcf_sort_segmented(to_dev(keys), to_dev(offsets.view(np.int64)), to_dev(vals),
                                  ws=ws)
    np.testing.assert_array_equal(to_host(gk, np.float64), rk)
    np.testing.assert_array_equal(to_host(gv, np.uint32), rv)
    x = torch.from_numpy(datagen.f64("lognormal", 40_000_000, 53)).to("cuda")
    got = P.sort(x)
    ref, _ = torch.sort(x)
    assert torch.equal(got, ref)
