"""Point-mass inputs (the robustness experiment of App. C): n keys plus n
copies of one in-range value.  The sorted output and the argsort (ties by
position, which the n equal keys make visible) match the oracle; at a large
size they match the library sort, and the profile attributes the point mass
to the single-value exits."""
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


@pytest.mark.parametrize("dist", ["normal", "uniform", "lognormal"])
def test_point_mass_matches_oracle(P, oracle, dist):
    banner(f"adversarial {dist} 2 x 300000")
    x = datagen.adversarial(dist, 300_000, 71)
    ref, ridx, _ = oracle.argsort(x)
    d = to_dev(x)
    np.testing.assert_array_equal(to_host(P.sort(d), np.float64), ref)
    k, i = P.pcf_argsort(d)
    np.testing.assert_array_equal(to_host(k, np.float64), ref)
    np.testing.assert_array_equal(to_host(i, np.uint32), ridx)


def test_point_mass_large_and_profiled(P):
    import torch
    banner("adversarial normal 2 x 2e7")
    n = 20_000_000
    x = datagen.adversarial("normal", n, 72)
    d = to_dev(x)
    P.pcf_profile_enable(True)
    P.pcf_profile_read(reset=True)
    got = P.sort(d)
    torch.cuda.synchronize()
    prof = P.pcf_profile_read(reset=True)
    P.pcf_profile_enable(False)
    ref, _ = torch.sort(d)
    assert torch.equal(got, ref)
    # the n copies of the point mass end in single-valued arrays
    assert prof["single_keys"]["keys"] >= n
