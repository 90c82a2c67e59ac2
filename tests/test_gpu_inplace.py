"""The in-place variant (keys sorted within their own array) on the GPU.

Below the staging capacity (2^24 keys) an array goes through the staging
buffer; above it the nodes are bucketed in place by the model (eight rounds
of two-way in-place partitions) before their buckets are staged.  Outputs are
compared with the CPU oracle (small sizes) and with torch's sort (large
sizes); the workspace stays far below a copy of the keys."""
import numpy as np
import pytest

from paper_2405_07122_amd import datagen
from tests.gpu_util import banner, to_dev, to_host

pytestmark = pytest.mark.gpu

STAGE = 1 << 24


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2405_07122_amd import pcfsort
    pcfsort.load()
    return pcfsort


@pytest.mark.parametrize("n", [0, 1, 99, 5000, 1_000_003])
def test_inplace_small_vs_oracle(P, oracle, n):
    banner(f"in place, staged, n={n}")
    x = datagen.f64("lognormal", n, 500 + n)
    d = to_dev(x)
    P.pcf_sort_inplace(d)
    ref, _, _ = oracle.sort(x)
    np.testing.assert_array_equal(to_host(d, np.float64), ref)


def _u64_check(P, x):
    import torch
    d = to_dev(x)
    flip = torch.tensor(-(2**63), dtype=torch.int64, device="cuda")
    ref, _ = torch.sort(d ^ flip)
    P.pcf_sort_inplace(d)
    assert torch.equal(d ^ flip, ref)


CASES = [
    ("normal", lambda n: datagen.f64("normal", n, 61)),
    ("mix8", lambda n: datagen.f64("mix8", n, 62)),
    ("point_mass", lambda n: datagen.adversarial("exponential", n // 2, 63)),
    ("two_valued", lambda n: np.where(np.random.default_rng(64).random(n) < 0.3, 1.25, -7.5)),
    ("nested_scales", lambda n: datagen.nested_scales(n, 65)),
]


@pytest.mark.parametrize("name,gen", CASES, ids=[c[0] for c in CASES])
def test_inplace_large_f64(P, name, gen):
    import torch
    n = 3 * STAGE + 12_345
    banner(f"in place f64 {name} n={n}")
    x = gen(n)
    d = to_dev(x)
    ref, _ = torch.sort(d)
    P.pcf_sort_inplace(d)
    assert torch.equal(d, ref)
    # the workspace holds no copy of the keys: a fixed part (the staging buffer
    # and its sort workspace) plus less than 1/32 of the key bytes, and less
    # than the out-of-place workspace
    w1, w4 = P.inplace_workspace_bytes(P.KEY_F64, n), P.inplace_workspace_bytes(P.KEY_F64, 4 * n)
    assert w4 - w1 < 3 * n * 8 // 32
    assert w1 < P.workspace_bytes(P.KEY_F64, n)


@pytest.mark.parametrize("kind", datagen.U64_KINDS)
def test_inplace_large_u64(P, kind):
    n = 2 * STAGE + 777
    banner(f"in place u64 {kind} n={n}")
    _u64_check(P, datagen.u64(kind, n, 66, distinct=10_000))


def test_inplace_invalid_key_and_errors(P):
    import torch
    banner("in place: invalid key, arguments")
    n = STAGE + 5000
    x = datagen.f64("uniform", n, 67)
    x[n - 3] = np.nan
    d = to_dev(x)
    with pytest.raises(P.PcfError) as e:
        P.pcf_sort_inplace(d)
    assert e.value.code == P.ERR_INVALID_KEY
    small = torch.zeros(16, dtype=torch.float64, device="cuda")
    ws = torch.empty(16, dtype=torch.uint8, device="cuda")
    with pytest.raises(P.PcfError) as e:
        P.pcf_sort_inplace(small, ws=ws)
    assert e.value.code == P.ERR_OUT_OF_MEMORY
