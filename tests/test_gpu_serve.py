"""Serving on the GPU: continuous batching gives every request the same bytes
it gets alone (through the server and through the plain call), argsort
positions included, under the HBM budget; a request with invalid keys fails
alone; the budget bounds what the server holds."""
import time

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


def _requests(count, seed, lo=8.0, hi=20.0):
    rng = np.random.default_rng(seed)
    out = []
    for j in range(count):
        n = int(np.floor(2 ** rng.uniform(lo, hi)))
        if rng.random() < 0.5:
            x = datagen.f64(datagen.F64_DISTS[j % 6], n, seed * 1000 + j)
        else:
            x = datagen.u64(datagen.U64_KINDS[j % 3], n, seed * 1000 + j, distinct=3000)
        out.append((x, bool(rng.random() < 0.5)))
    return out


def _plain(P, d, argsort):
    if argsort:
        k, i = P.pcf_argsort(d)
        return k, i
    return P.sort(d), None


def test_mix_equals_alone(P, oracle):
    import torch
    banner("serve: mix vs alone")
    reqs = _requests(48, 61)
    devs = [to_dev(x) for x, _ in reqs]
    with P.Server(hbm_budget_bytes=8 << 30, max_streams=3, max_batch_requests=32) as srv:
        # alone: one request at a time through the server
        alone = []
        for d, (x, a) in zip(devs[:8], reqs[:8]):
            t = srv.submit(d, argsort=a)
            r = srv.wait(t)
            assert r["status"] == 0 and r["batch_requests"] == 1
            alone.append((r["keys"].clone(), None if r["idx"] is None else r["idx"].clone()))
            srv.release(t)
        # the mix: everything submitted at once
        tickets = [srv.submit(d, argsort=a) for d, (x, a) in zip(devs, reqs)]
        batched = 0
        for j, (t, d, (x, a)) in enumerate(zip(tickets, devs, reqs)):
            r = srv.wait(t)
            assert r["status"] == 0, (j, r["status"])
            batched += r["batch_requests"] > 1
            pk, pi = _plain(P, d, a)
            assert torch.equal(r["keys"], pk), j
            if a:
                assert torch.equal(r["idx"], pi), j
            else:
                assert r["idx"] is None
            if j < 8:
                assert torch.equal(r["keys"], alone[j][0])
                if a:
                    assert torch.equal(r["idx"], alone[j][1])
            if j % 6 == 0:  # and the oracle, on a subset
                dt = np.float64 if x.dtype == np.float64 else np.uint64
                if a:
                    ok, oi, _ = oracle.argsort(x)
                    np.testing.assert_array_equal(to_host(r["idx"], np.uint32), oi)
                else:
                    ok, _, _ = oracle.sort(x)
                np.testing.assert_array_equal(to_host(r["keys"], dt), ok)
            srv.release(t)
        assert batched > 0  # requests that met in the queue shared a launch chain
        st = srv.stats()
        assert st["budget_in_use"] == 0 and st["budget_high_water"] <= st["budget_bytes"]
        assert st["completed"] == 56 and st["batches"] < 56


def test_budget_and_invalid_key(P):
    import torch
    banner("serve: budget, invalid key, shutdown")
    budget = 64 << 20
    with P.Server(hbm_budget_bytes=budget, max_streams=2, max_batch_requests=16) as srv:
        big = torch.rand(4_000_000, dtype=torch.float64, device="cuda")
        with pytest.raises(P.PcfError) as ei:
            srv.submit(big)
        assert ei.value.code == P.ERR_OUT_OF_MEMORY
        rng = np.random.default_rng(62)
        arrs = [rng.random(int(rng.integers(1000, 200_000))) for _ in range(24)]
        arrs[5][123] = np.nan
        devs = [to_dev(a) for a in arrs]
        ts = [srv.submit(d) for d in devs]
        for j, (t, a) in enumerate(zip(ts, arrs)):
            r = srv.wait(t)
            if j == 5:
                assert r["status"] == P.ERR_INVALID_KEY
            else:
                assert r["status"] == 0
                np.testing.assert_array_equal(to_host(r["keys"], np.float64), np.sort(a))
            st = srv.stats()
            assert st["budget_in_use"] <= budget
            srv.release(t)
        st = srv.stats()
        assert st["budget_high_water"] <= budget and st["budget_in_use"] == 0
        # results not released are freed by close(); pending ones finish first
        for d in devs[:4]:
            srv.submit(d)
    time.sleep(0.01)


def test_large_requests(P):
    """Requests from the top of the serving size range (2^21 .. 2^26 keys), fp64
    and uint64, keys only and argsort, submitted together: every result equals
    torch's (stable) sort of the request."""
    import torch
    banner("serve: large requests")
    sizes = [(1 << 21) + 3, (1 << 23) + 5, (1 << 24) - 7, (1 << 25) + 11, (1 << 26) - 1]
    rng = np.random.default_rng(77)
    reqs = []
    for j, m in enumerate(sizes):
        if j % 2 == 0:
            x = datagen.f64(datagen.F64_DISTS[j], m, 900 + j)
        else:
            x = datagen.u64(datagen.U64_KINDS[j % 3], m, 900 + j, distinct=50_000)
        reqs.append((to_dev(x), bool(rng.random() < 0.5) or j == 4))
    flip = torch.tensor(-(2**63), dtype=torch.int64, device="cuda")
    with P.Server(hbm_budget_bytes=16 << 30, max_streams=2, max_batch_requests=8,
                  max_batch_keys=1 << 28) as srv:
        tickets = [srv.submit(d, argsort=a) for d, a in reqs]
        for (d, a), t in zip(reqs, tickets):
            r = srv.wait(t)
            assert r["status"] == 0
            if d.dtype == torch.float64:
                rk, ri = torch.sort(d, stable=True)
                assert torch.equal(r["keys"], rk)
            else:
                rk, ri = torch.sort(d ^ flip, stable=True)
                assert torch.equal(r["keys"] ^ flip, rk)
            if a:
                assert torch.equal(r["idx"].to(torch.int64), ri)
            srv.release(t)
