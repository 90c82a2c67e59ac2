"""The CPU oracle against what the paper and the mathematics fix (no GPU)."""
import json
import math
import os
import sys

import numpy as np
import pytest

from tests import oracle_pins as P

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.mark.parametrize("pin", P.ALL_PINS, ids=lambda f: f.__name__)
def test_pin(oracle, pin):
    fails = pin(oracle, oracle.load())
    assert not fails, "\n".join(fails)


def test_splitmix64_published_vectors(oracle):
    g = json.load(open(os.path.join(GOLDEN, "splitmix64_vectors.json")))
    got0 = [oracle.splitmix64(0, k) for k in range(5)]
    assert got0 == [int(h, 16) for h in g["seed_0"]]
    got1 = [oracle.splitmix64(1234567, k) for k in range(5)]
    assert got1 == g["seed_1234567"]


def test_sample_positions_uniform(oracle):
    """Samples are uniform draws with replacement over [0, n) (Sec. 3.3 and the
    independence used in the proofs): a chi-square test on 64 position bins."""
    n, alpha = 1_000_003, 200_000
    x = np.arange(n, dtype=np.float64)
    lv = oracle.level(x, alpha, 10, 10, oracle.node_seed(3, 0, 0, 0))
    counts = np.bincount((lv.sample_pos * 64 // n).astype(np.int64), minlength=64)
    exp = alpha / 64.0
    chi2 = float(((counts - exp) ** 2 / exp).sum())
    assert chi2 < 120.0  # 63 dof: p < 1e-5 beyond this
    assert lv.sample_pos.max() < n


def test_root34_exact(oracle):
    """floor(n^{3/4}) (Sec. 3.3 theorems) against exact integer arithmetic."""
    g = json.load(open(os.path.join(GOLDEN, "paper_parameters.json")))
    p, q = g["exponent_num"], g["exponent_den"]
    rng = np.random.default_rng(0)
    ns = [1, 2, 15, 16, 81, 100, 4096, 10**6, 10**8, 2 * 10**8, 2**40] + list(
        rng.integers(1, 2**40, size=200))
    for n in ns:
        n = int(n)
        m = oracle.root34(n)
        assert m ** q <= n ** p < (m + 1) ** q, n


def test_paper_quantization_example(oracle):
    """App. A.4: for the whole fp64 range, eta = 1.99e292, |I| = 3.59e308,
    eta/|I| = 5.55e-17, so the condition holds for beta up to ~9e15."""
    g = json.load(open(os.path.join(GOLDEN, "paper_quantization_example.json")))
    dmax = sys.float_info.max
    eta = oracle.eta_f64(-dmax, dmax)
    ratio = oracle.quant_lhs_f64(1, -dmax, dmax)

    def sig3(v):
        return float(f"{v:.3g}")

    assert sig3(eta) == g["eta"] or abs(eta / g["eta"] - 1) < 5e-3
    # |I| = 2 * DBL_MAX is not representable in fp64; compare as decimals
    from decimal import Decimal
    assert abs(2 * Decimal(dmax) / Decimal(g["interval_width"]) - 1) < Decimal("5e-3")
    assert sig3(ratio) == g["ratio"]
    assert abs((0.5 / ratio) / g["beta_limit"] - 1) < 0.01
    # the condition at the limit is exactly the threshold 1/2 for beta = 2^53
    assert oracle.quant_lhs_f64(2**53, -dmax, dmax) <= 0.5
    assert oracle.quant_lhs_f64(2**53 + 2**40, -dmax, dmax) > 0.5


def test_special_cases(oracle):
    # n < tau: the standard sort alone (Algorithm 1, small-array branch)
    x = np.array([3.0, 1.0, 2.0])
    s, _, st = oracle.sort(x)
    assert list(s) == [1.0, 2.0, 3.0] and st["levels"] == 0 and st["small_sorts"] == 1
    # all equal: single-value early exit (Sec. 4.1)
    x = np.full(5000, 7.25)
    s, idx, st = oracle.argsort(x)
    assert np.array_equal(s, x) and np.array_equal(idx, np.arange(5000)) and st["single_valued"] == 1
    # empty and one key
    assert oracle.sort(np.zeros(0))[0].shape == (0,)
    assert list(oracle.sort(np.array([4.0]))[0]) == [4.0]
    # sorted, reverse sorted, two-valued
    rng = np.random.default_rng(1)
    u = np.sort(rng.random(50_000))
    for x in (u, u[::-1].copy(), np.where(rng.random(50_000) < 0.3, 1.0, 2.0)):
        s, idx, _ = oracle.argsort(x)
        assert np.array_equal(s, np.sort(x))
        assert np.array_equal(idx, np.argsort(x, kind="stable"))


def test_invalid_keys(oracle):
    for bad in (np.nan, np.inf, -np.inf, -0.0):
        x = np.array([1.0, 2.0, bad, 3.0] * 50)
        with pytest.raises(oracle.OracleError) as e:
            oracle.sort(x)
        assert e.value.code == oracle.ERR_INVALID_KEY


def test_overflowing_range_uses_halves(oracle):
    dmax = sys.float_info.max
    rng = np.random.default_rng(4)
    x = np.concatenate([[-dmax, dmax], rng.uniform(-1, 1, 5000) * dmax * 0.9, rng.random(500)])
    lv = oracle.level(x, 300, 300, 300, 5, vals=np.arange(x.shape[0], dtype=np.uint32))
    assert lv.halves == 1 and lv.status == 0
    s, idx, _ = oracle.argsort(x)
    assert np.array_equal(s, np.sort(x))


def test_nonfinite_scale_is_a_failure(oracle):
    """A range of a few subnormals makes beta / (x_max - x_min) overflow: the node
    is sorted by the standard sort (reading of the worst-case exception rule)."""
    tiny = np.array([5e-324, 1e-323, 1.5e-323, 2e-323])
    x = np.tile(tiny, 100)[np.random.default_rng(0).permutation(400)]
    s, _, st = oracle.sort(x)
    assert st["nonfinite_scale"] >= 1
    assert np.array_equal(s, np.sort(x))


def test_u64_extremes(oracle):
    top = np.uint64(2**64 - 1)
    rng = np.random.default_rng(8)
    x = np.concatenate([np.array([0, top, top, 1], dtype=np.uint64),
                        rng.integers(0, 2**64 - 1, 20_000, dtype=np.uint64, endpoint=True)])
    s, idx, _ = oracle.argsort(x)
    assert np.array_equal(s, np.sort(x))
    assert np.array_equal(idx, np.argsort(x, kind="stable"))


def test_quantization_condition_holds(oracle):
    """The fine-enough-quantization condition (App. A.4) on synthetic data."""
    _, _, st = oracle.sort(np.random.default_rng(0).standard_normal(300_000))
    assert 0.0 < st["max_quant_lhs"] <= 0.5


def test_point_mass_input(oracle):
    """The oracle on the point-mass input of App. C: sorted like the library
    sort, with the point mass leaving through the single-value exit (or the
    standard sort of a failed bucket) rather than by endless recursion."""
    from paper_2405_07122_amd import datagen
    x = datagen.adversarial("normal", 20_000, 5)
    out, _, st = oracle.sort(x)
    np.testing.assert_array_equal(out, np.sort(x))
    assert st["single_valued"] + st["fail_sorts"] >= 1
    assert st["max_depth"] <= 6
