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
        # rep_n is what the class was timed on (for the small classes a
        # segmented batch larger than the class); look the class up by its range
        for n in (max(e["min_n"], 1), e["max_n"] - 1):
            assert P.policy_for(P.KEY_F64, n) == e["policy"], (n, e)
    for n, dist in [(300_001, "lognormal"), (5_000_000, "mix8"), (40_000_000, "normal")]:
        x = datagen.f64(dist, n, 77)
        d = to_dev(x)
        got = P.sort(d)
        ref, _ = torch.sort(d)
        assert torch.equal(got, ref), (n, dist)
        if n <= 300_001:
            np.testing.assert_array_equal(to_host(got, np.float64), oracle.sort(x)[0])
    P.pcf_load_tuning(None)


def test_node_parameters_by_size_class(P, oracle, tmp_path):
    """A loaded table drives every global node by its own length: a segmented
    batch with a payload (graph path) and a plain sort under four classes with
    different buckets, samples, bins, chunk sizes and scatter tiles stay
    bit-exact to the oracle, and the workspace query covers every class."""
    import torch
    banner("per-node policies from a tuning table")
    classes = [(0, 1 << 14, 64, 8, 8, 8192, 1024), (1 << 14, 1 << 18, 128, 32, 16, 16384, 2048),
               (1 << 18, 1 << 22, 512, 16, 32, 8192, 1024), (1 << 22, 1 << 32, 256, 16, 16, 32768, 2048)]
    base = P.get_policy()
    ents = []
    for lo, hi, mb, sp, bp, ck, tile in classes:
        pol = dict(base, max_buckets=mb, samples_per_bucket=sp, bins_per_bucket=bp, chunk_keys=ck,
                   scatter_tile=tile)
        ents.append({"key_type": 0, "with_payload": 1, "min_n": lo, "max_n": hi, "policy": pol})
    path = tmp_path / "classes.json"
    path.write_text(json.dumps({"format": "pcfsort-tuning-1", "entries": ents}))
    n_ref = P.workspace_bytes(P.KEY_F64, 3_000_000, True, 64)
    P.pcf_load_tuning(str(path))
    try:
        assert P.workspace_bytes(P.KEY_F64, 3_000_000, True, 64) >= n_ref
        keys, offsets, vals = datagen.segments(num=64, lo_log2=8, hi_log2=21, seed=41)
        n = int(offsets[-1])
        ws = P.workspace(P.KEY_F64, n, True, 64)
        st = torch.zeros(1, dtype=torch.int32, device="cuda")
        for rep in range(2):
            gk, gv = P.pcf_sort_segmented(to_dev(keys), to_dev(offsets.view(np.int64)), to_dev(vals),
                                          ws=ws, d_status=st)
            torch.cuda.synchronize()
            assert int(st.cpu()[0]) == 0
        ref_k, ref_v = oracle.sort_segmented(keys, offsets, vals)
        np.testing.assert_array_equal(to_host(gk, np.float64), ref_k)
        np.testing.assert_array_equal(to_host(gv, np.uint32), ref_v)
        x = datagen.f64("lognormal", 2_500_000, 43)
        k, i = P.pcf_argsort(to_dev(x))
        rk, ri, _ = oracle.argsort(x)
        np.testing.assert_array_equal(to_host(k, np.float64), rk)
        np.testing.assert_array_equal(to_host(i, np.uint32), ri)
    finally:
        P.pcf_load_tuning(None)
        P.pcf_graph_clear()
