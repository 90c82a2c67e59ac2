"""Autotuner on the GPU: it writes a valid table for every size class, the
table loads, and sorts under the tuned policies stay bit-exact."""
import json

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
    yield pcfsort
    pcfsort.pcf_load_tuning(None)


def test_autotune_roundtrip(P, oracle, tmp_path):
    import torch
    banner("autotune f64 keys only")
    out = tmp_path / "tune.json"
    P.pcf_autotune(P.KEY_F64, False, str(out))
    t = json.loads(out.read_text())
    assert t["format"] == "pcfsort-tuning-1" and len(t["entries"]) == 4
    for e in t["entries"]:
        assert e["ms_per_sort"] > 0 and e["policy"]["max_buckets"] in (64, 128, 256, 512)
    P.pcf_load_tuning(str(out))
    for e in t["entries"]:
        assert P.policy_for(P.KEY_F64, e["rep_n"])["max_buckets"] == e["policy"]["max_buckets"]
    for n, dist in [(300_001, "lognormal"), (5_000_000, "mix8"), (40_000_000, "normal")]:
        x = datagen.f64(dist, n, 77)
        d = to_dev(x)
        got = P.sort(d)
        ref, _ = torch.sort(d)
        assert torch.equal(got, ref), (n, dist)
        if n <= 300_001:
            np.testing.assert_array_equal(to_host(got, np.float64), oracle.sort(x)[0])
    P.pcf_load_tuning(None)
