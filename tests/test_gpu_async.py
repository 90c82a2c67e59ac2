"""Calls that only enqueue (a device status word is given: a fixed chain of
levels, no host read) and calls that wait (the host reads the control block
after the planned levels).

- An input that needs more global levels than the delta rule plans (multi-
  scale u64 clusters take radix levels): a waiting call runs a second
  LDS-finish pass for the items of those levels, an enqueue-only call runs
  them inside its chain; the output matches the oracle both ways.
- Profile figures of calls that only enqueue are folded in at
  pcf_profile_read; they count the same keys per kernel as calls that wait
  (the chain's empty levels add launches, not keys).
- A data error reaches the status word of a call given one."""
import numpy as np
import pytest

from paper_2405_07122_amd import datagen
from tests.gpu_util import banner, to_dev, to_host

pytestmark = pytest.mark.gpu

LDS_CAP = 8192


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2405_07122_amd import pcfsort
    pcfsort.load()
    return pcfsort


def _root34(m: int) -> int:
    """floor(m^{3/4}) exactly: the largest r with r^4 <= m^3."""
    r = int(round(m ** 0.75))
    while r ** 4 > m ** 3:
        r -= 1
    while (r + 1) ** 4 <= m ** 3:
        r += 1
    return r


def _planned_levels(n: int) -> int:
    d, m = 0, n
    while m > LDS_CAP:
        m = _root34(m)
        d += 1
    return d


def test_extra_levels_take_a_second_finish_pass(P, oracle):
    import torch
    n = 3_000_000
    banner(f"u64 clustered n={n}: levels beyond the plan")
    x = datagen.u64("clustered", n, 8)
    ref, _, _ = oracle.sort(x)
    d = to_dev(x)
    P.pcf_profile_select(None)
    P.pcf_profile_enable(True)
    P.pcf_profile_read(reset=True)
    got = P.pcf_sort_u64(d)
    prof = P.pcf_profile_read(reset=True)
    P.pcf_profile_enable(False)
    np.testing.assert_array_equal(to_host(got, np.uint64), ref)
    levels = prof["scatter"]["launches"]
    assert levels > _planned_levels(n)  # multi-scale clusters need radix levels
    assert prof["lds_small"]["launches"] == 2  # one pass after the plan, one after the rest
    # the same call that only enqueues
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    out = torch.empty_like(d)
    P.pcf_sort_u64(d, out=out, d_status=st)
    torch.cuda.synchronize()
    assert int(st.item()) == 0
    np.testing.assert_array_equal(to_host(out, np.uint64), ref)


def test_deferred_profile_equals_waiting_profile(P):
    # argsort: its scatters are stable, so every call builds the same
    # recursion and the figures of the two modes must agree exactly (keys
    # alone may sit in any order inside a bucket, so the samples of deeper
    # levels, and the arrays they produce, can differ from call to call)
    import torch
    n = 2_000_000
    banner(f"profile of enqueue-only calls, n={n}")
    d = to_dev(datagen.f64("normal", n, 2))
    ko = torch.empty_like(d)
    io = torch.empty(n, dtype=torch.int32, device="cuda")
    ws = P.workspace(P.KEY_F64, n, with_payload=True)
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    P.pcf_profile_select(None)
    P.pcf_profile_enable(True)
    figs = []
    for status in (None, st):
        P.pcf_profile_read(reset=True)
        for _ in range(3):
            P.pcf_argsort(d, keys_out=ko, idx_out=io, ws=ws, d_status=status)
        torch.cuda.synchronize()
        figs.append(P.pcf_profile_read(reset=True))
    P.pcf_profile_enable(False)
    assert int(st.item()) == 0
    wait, enq = figs
    for k in wait:
        assert enq[k]["launches"] >= wait[k]["launches"], k
        assert wait[k]["keys"] == enq[k]["keys"], k
        if wait[k]["launches"]:
            assert enq[k]["ms"] > 0, k
    assert enq["scatter"]["launches"] >= 3


def test_status_word_of_enqueue_only_call(P):
    import torch
    banner("invalid key, enqueue-only call")
    x = datagen.f64("uniform", 1_000_000, 5)
    x[777] = np.nan
    st = torch.zeros(1, dtype=torch.int32, device="cuda")
    d = to_dev(x)
    # the error reaches the status word; the call itself returns after enqueue
    P.pcf_sort_f64(d, d_status=st)
    torch.cuda.synchronize()
    assert int(st.item()) == P.ERR_INVALID_KEY
    # and a valid input afterwards clears it
    P.pcf_sort_f64(to_dev(datagen.f64("uniform", 1_000_000, 6)), d_status=st)
    torch.cuda.synchronize()
    assert int(st.item()) == 0
