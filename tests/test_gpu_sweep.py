"""A seeded sweep of sizes and input structures through the plain, argsort
and segmented calls.

Sizes sit on and around the boundaries of the GPU's tiles, work units and
LDS classes (and the tau and LDS-capacity thresholds); inputs include sorted
and reversed runs, all-equal and two-valued arrays, heavy duplicates, tiny
and huge ranges, subnormals and u64 extremes.  The sorted output is unique,
so every result is compared element by element with the oracle (up to
200,000 keys) and with numpy's stable sort above that."""
import numpy as np
import pytest

from paper_2405_07122_amd import datagen
from tests.gpu_util import banner, to_dev, to_host

pytestmark = pytest.mark.gpu

SIZES = [1, 2, 3, 99, 100, 101, 255, 256, 257, 2047, 2048, 2049, 4095, 4096, 4097, 8191, 8192,
         8193, 12288, 16383, 16384, 16385, 24413, 24415, 32769, 65537, 131071, 200_003, 262145,
         1_000_003, 3_000_017]
ORACLE_MAX = 200_000


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2405_07122_amd import pcfsort
    pcfsort.load()
    return pcfsort


def _f64_input(kind: str, n: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    if kind == "sorted":
        x = np.sort(datagen.f64("normal", n, seed))
    elif kind == "reversed":
        x = np.sort(datagen.f64("exponential", n, seed))[::-1].copy()
    elif kind == "equal":
        x = np.full(n, 2.5)
    elif kind == "two":
        x = np.where(rng.random(n) < 0.3, -1.0, 7.0)
    elif kind == "dups":
        x = np.round(datagen.f64("normal", n, seed) * 4) / 4 + 0.0
    elif kind == "tiny_range":
        x = 1.0 + rng.integers(0, 1000, n) * np.finfo(np.float64).eps
    elif kind == "huge_range":
        x = rng.choice(np.array([-1e308, -1e300, -1.0, 0.0, 1e-300, 1.0, 1e300, 1e308]), n)
        x = x * (1.0 + rng.random(n) * 1e-3) + 0.0
        x = np.clip(x, -np.finfo(np.float64).max, np.finfo(np.float64).max)
    elif kind == "subnormal":
        x = rng.integers(0, 1 << 40, n).astype(np.uint64).view(np.float64).copy()
    else:
        x = datagen.f64(kind, n, seed)
    return np.ascontiguousarray(x, dtype=np.float64)


def _u64_input(kind: str, n: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    if kind == "extremes":
        return rng.choice(np.array([0, 1, 2**63 - 1, 2**63, 2**64 - 2, 2**64 - 1], dtype=np.uint64), n)
    if kind == "full":
        return rng.integers(0, 2**64 - 1, n, dtype=np.uint64, endpoint=True)
    return datagen.u64(kind, n, seed, distinct=max(2, n // 50))


def _check(got: np.ndarray, x: np.ndarray, oracle, argsort_idx=None):
    if x.shape[0] <= ORACLE_MAX:
        if argsort_idx is None:
            ref, _, _ = oracle.sort(x)
        else:
            ref, ridx, _ = oracle.argsort(x)
            np.testing.assert_array_equal(argsort_idx, ridx)
    else:
        order = np.argsort(x, kind="stable")
        ref = x[order]
        if argsort_idx is not None:
            np.testing.assert_array_equal(argsort_idx, order.astype(np.uint32))
    np.testing.assert_array_equal(got, ref)


F64_KINDS = list(datagen.F64_DISTS) + ["sorted", "reversed", "equal", "two", "dups", "tiny_range",
                                      "huge_range", "subnormal"]


@pytest.mark.parametrize("n", SIZES)
def test_sweep_f64_keys_and_argsort(P, oracle, n):
    kinds = F64_KINDS[(n % 7)::3]  # a rotating subset per size
    for j, kind in enumerate(kinds):
        banner(f"sweep f64 {kind} n={n}")
        x = _f64_input(kind, n, 1000 * n % 9973 + j)
        d = to_dev(x)
        _check(to_host(P.sort(d), np.float64), x, oracle)
        if j == 0 or n <= 100_000:
            k, i = P.pcf_argsort(d)
            _check(to_host(k, np.float64), x, oracle, to_host(i, np.uint32))


@pytest.mark.parametrize("n", [n for n in SIZES if n >= 100])
def test_sweep_u64(P, oracle, n):
    for j, kind in enumerate(["extremes", "full"] + list(datagen.U64_KINDS)):
        if (n + j) % 2:
            continue
        banner(f"sweep u64 {kind} n={n}")
        x = _u64_input(kind, n, n + j)
        _check(to_host(P.pcf_sort_u64(to_dev(x)), np.uint64), x, oracle)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_sweep_segmented(P, seed):
    import torch
    rng = np.random.default_rng(seed)
    nseg = int(rng.integers(1, 400))
    sizes = np.where(rng.random(nseg) < 0.15, 0,
                     np.floor(np.exp2(rng.uniform(0, 17, nseg)))).astype(np.int64)
    offsets = np.zeros(nseg + 1, dtype=np.uint64)
    offsets[1:] = np.cumsum(sizes)
    n = int(offsets[-1])
    banner(f"sweep segmented seed={seed} segments={nseg} n={n}")
    x = np.concatenate([_f64_input(F64_KINDS[s % len(F64_KINDS)], int(sizes[s]), seed * 1000 + s)
                        for s in range(nseg)]) if n else np.zeros(0)
    vals = np.concatenate([np.arange(int(sz), dtype=np.uint32) for sz in sizes]) if n else \
        np.zeros(0, dtype=np.uint32)
    dk = to_dev(x)
    dv = to_dev(vals)
    doff = torch.from_numpy(offsets.view(np.int64)).to("cuda")
    for ws in (None, P.workspace(P.KEY_F64, max(n, 1), True, nseg)):
        ko, vo = P.pcf_sort_segmented(dk, doff, dv, ws=ws)
        gk, gv = to_host(ko, np.float64), to_host(vo, np.uint32)
        for s in range(nseg):
            a, b = int(offsets[s]), int(offsets[s + 1])
            order = np.argsort(x[a:b], kind="stable")
            np.testing.assert_array_equal(gk[a:b], x[a:b][order])
            np.testing.assert_array_equal(gv[a:b], vals[a:b][order])
