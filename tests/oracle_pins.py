"""Pins that tie the CPU oracle to what the paper and the mathematics fix.

Each pin takes the oracle's Python front end and a loaded library handle and
returns a list of failure messages (empty = pinned).  test_oracle_pins.py runs
them against the real oracle; test_oracle_plants.py builds copies of the
oracle with deliberate mistakes compiled in and checks that every mistake
trips at least one pin.  None of these pins retypes the oracle's formulas: they
use library sorts, brute force, closed forms, invariants and the paper's
bound on bucketing failures.
"""
from __future__ import annotations

import itertools
import math

import numpy as np

from paper_2405_07122_amd import datagen


def _np_stable_argsort(x):
    return np.argsort(x, kind="stable").astype(np.uint32)


def pin_library_sort(O, lib) -> list[str]:
    """The output is the unique ascending order (problem statement, Sec. 3.1):
    equal to numpy's sort; the payload order equals numpy's stable argsort."""
    fails = []
    cases = []
    for d in datagen.F64_DISTS:
        cases.append((d, datagen.f64(d, 30_000, 100 + len(cases))))
    for k in datagen.U64_KINDS:
        cases.append((k, datagen.u64(k, 30_000, 200 + len(cases), distinct=300)))
    # heavy duplicates in fp64: two decimals of a normal draw
    cases.append(("dup_f64", np.round(datagen.f64("normal", 40_000, 7), 2) + 0.0))
    for name, x in cases:
        s, idx, _ = O.argsort(x, lib=lib)
        if not np.array_equal(s, np.sort(x, kind="stable")):
            fails.append(f"{name}: keys differ from numpy sort")
        if not np.array_equal(idx, _np_stable_argsort(x)):
            fails.append(f"{name}: argsort differs from numpy stable argsort")
    return fails


def pin_brute_force(O, lib) -> list[str]:
    """Every permutation of small multisets, learned path forced on (tau = 2)."""
    fails = []
    bases = [[0.5, 1.5, 2.5, 3.5, 4.5, 5.5], [1.0, 1.0, 2.0, 2.0, 3.0, 7.0], [3.0, 3.0, 3.0, 1.0, 9.0, 9.0, 2.0]]
    for base in bases:
        seen = set()
        for perm in itertools.permutations(range(len(base))):
            x = np.array([base[p] for p in perm], dtype=np.float64)
            key = x.tobytes()
            if key in seen:
                continue
            seen.add(key)
            s, idx, _ = O.argsort(x, tau=2, lib=lib)
            want = sorted(range(len(x)), key=lambda i: (x[i], i))
            if list(idx) != want or list(s) != [x[i] for i in want]:
                fails.append(f"permutation {perm} of {base}: got {list(idx)} want {want}")
                break
    return fails


def pin_selection_sort(O, lib) -> list[str]:
    """An O(n^2) selection sort written here, n <= 600, tau in {2, 100}."""
    fails = []
    rng = np.random.default_rng(5)
    for n in (1, 2, 3, 17, 99, 100, 101, 257, 600):
        x = np.round(rng.standard_normal(n) * 4.0) / 4.0 + 0.0
        ref = list(x)
        for i in range(n):
            m = i
            for j in range(i + 1, n):
                if ref[j] < ref[m]:
                    m = j
            ref[i], ref[m] = ref[m], ref[i]
        for tau in (2, 100):
            s, _, _ = O.sort(x, tau=tau, lib=lib)
            if list(s) != ref:
                fails.append(f"n={n} tau={tau}: differs from selection sort")
    return fails


def _check_level(name, x, lv, alpha, beta, gamma, with_vals=True) -> list[str]:
    """Invariants of one bucketing (Sec. 3.3 and the contiguity remark of Sec. 3.2)."""
    fails = []
    b, T, sizes = lv.b.astype(np.int64), lv.T.astype(np.int64), lv.sizes.astype(np.int64)
    if np.any(np.diff(b) < 0) or b[0] < 0:
        fails.append(f"{name}: b not non-decreasing and non-negative")
    if b[beta] != alpha:
        fails.append(f"{name}: b[beta] = {b[beta]} != alpha = {alpha}")
    if np.any(np.diff(T) < 0) or T[0] < 0 or T[beta] != gamma:
        fails.append(f"{name}: T not non-decreasing in [0, gamma] with T[beta] = gamma")
    if sizes.sum() != x.shape[0]:
        fails.append(f"{name}: bucket sizes sum to {sizes.sum()} != n")
    part = lv.part_keys
    if not np.array_equal(np.sort(part), np.sort(x)):
        fails.append(f"{name}: partition is not a permutation of the input")
    bounds = np.concatenate([[0], np.cumsum(sizes)])
    prev_max = None
    for j in range(gamma + 1):
        seg = part[bounds[j]:bounds[j + 1]]
        if seg.size == 0:
            continue
        if prev_max is not None and not prev_max < seg.min():
            fails.append(f"{name}: bucket {j} overlaps an earlier bucket (contiguity)")
            break
        prev_max = seg.max()
    if with_vals and lv.part_vals is not None:
        for j in range(gamma + 1):
            v = lv.part_vals[bounds[j]:bounds[j + 1]]
            if np.any(np.diff(v.astype(np.int64)) <= 0):
                fails.append(f"{name}: bucket {j} not in input order (Append is in order)")
                break
    return fails


def pin_level_invariants(O, lib) -> list[str]:
    fails = []
    rng = np.random.default_rng(11)
    for name, x, (a, be, g) in [
        ("uniform", datagen.f64("uniform", 20_000, 3), (500, 800, 120)),
        ("lognormal", datagen.f64("lognormal", 20_000, 4), (1000, 300, 63)),
        ("dups", np.round(rng.standard_normal(20_000), 1) + 0.0, (700, 700, 700)),
        ("zipf", datagen.u64("zipf", 20_000, 5, distinct=500), (300, 4000, 255)),
        ("bursty", datagen.u64("bursty", 20_000, 6), (2000, 2000, 100)),
    ]:
        idx = np.arange(x.shape[0], dtype=np.uint32)
        lv = O.level(x, a, be, g, O.node_seed(1, 0, 0, 0, lib=lib), vals=idx, lib=lib)
        if lv.status != 0:
            fails.append(f"{name}: unexpected status {lv.status}")
            continue
        fails += _check_level(name, x, lv, a, be, g)
    return fails


def pin_identity_closed_form(O, lib) -> list[str]:
    """With x a permutation of 0..n-1, beta = n-1 and the whole array as the
    sample (alpha = n), i(x) = x exactly, so b_i = i + 1 and the bucket of key v
    is floor((v + 1) gamma / n): every count has a closed form (Sec. 3.3)."""
    fails = []
    rng = np.random.default_rng(2)
    for dtype in (np.float64, np.uint64):
        for n, gamma in ((1000, 37), (4096, 64), (777, 776)):
            v = rng.permutation(n)
            x = v.astype(dtype)
            lv = O.level(x, n, n - 1, gamma, 0, sample_idx=np.arange(n, dtype=np.uint64),
                         vals=np.arange(n, dtype=np.uint32), lib=lib)
            i = np.arange(n, dtype=np.int64)
            want_b = i + 1
            want_T = ((i + 1) * gamma) // n
            want_sizes = np.bincount(want_T, minlength=gamma + 1)
            tag = f"{np.dtype(dtype).name} n={n} gamma={gamma}"
            if not np.array_equal(lv.b.astype(np.int64), want_b):
                fails.append(f"{tag}: b differs from i + 1")
            if not np.array_equal(lv.T.astype(np.int64), want_T):
                fails.append(f"{tag}: T differs from floor((i + 1) gamma / n)")
            if not np.array_equal(lv.sizes.astype(np.int64), want_sizes):
                fails.append(f"{tag}: bucket sizes differ from the closed form")
            # bucket of key v is want_T[v]; the partition lists keys bucket by bucket, in input order
            order = np.argsort(want_T[v], kind="stable")
            if not np.array_equal(lv.part_keys, x[order]):
                fails.append(f"{tag}: partition differs from the stable closed form")
    return fails


def pin_halved_range_closed_form(O, lib) -> list[str]:
    """Keys k 2^(1023-m) for k = -2^m..2^m span [-2^1023, 2^1023], whose width
    overflows fp64, so the bin function works on halves (reading C11 of the
    Sec. 3.3 bin function).  With beta = 2^(m+1) the halved scale is exactly
    2^(m+1) / 2^1023 and the halved offset of key k is (k + 2^m) 2^(1022-m),
    so key k sits exactly at bin k + 2^m; with every key sampled once,
    b_i = i + 1.  Halving only one operand (v/2 - x_min, or v - x_min/2)
    moves every key by 2^m bins and breaks the closed form."""
    fails = []
    rng = np.random.default_rng(6)
    for m, reps, gamma in ((3, 1, 16), (3, 40, 5), (7, 3, 200), (10, 1, 63)):
        k = np.arange(-(2 ** m), 2 ** m + 1, dtype=np.int64)
        grid = k.astype(np.float64) * 2.0 ** (1023 - m)
        beta = 2 ** (m + 1)
        x = np.tile(grid, reps)[rng.permutation(grid.shape[0] * reps)] + 0.0
        n = x.shape[0]
        # one sample per distinct key: the first occurrence of each grid point
        first = {}
        for i, v in enumerate(x):
            first.setdefault(float(v), i)
        sidx = np.array([first[float(v)] for v in grid], dtype=np.uint64)
        alpha = sidx.shape[0]
        lv = O.level(x, alpha, beta, gamma, 0, sample_idx=sidx,
                     vals=np.arange(n, dtype=np.uint32), lib=lib)
        tag = f"m={m} reps={reps}"
        if lv.halves != 1:
            fails.append(f"{tag}: range width did not overflow into the halved form")
            continue
        i = np.arange(beta + 1, dtype=np.int64)
        want_b = i + 1
        want_T = ((i + 1) * gamma) // alpha
        if not np.array_equal(lv.b.astype(np.int64), want_b):
            fails.append(f"{tag}: b differs from i + 1")
        if not np.array_equal(lv.T.astype(np.int64), want_T):
            fails.append(f"{tag}: T differs from floor((i + 1) gamma / alpha)")
        kb = np.round(x / 2.0 ** (1023 - m)).astype(np.int64) + 2 ** m  # exact bin of each key
        want_sizes = np.bincount(want_T[kb], minlength=gamma + 1)
        if not np.array_equal(lv.sizes.astype(np.int64), want_sizes):
            fails.append(f"{tag}: bucket sizes differ from the closed form")
        order = np.argsort(want_T[kb], kind="stable")
        if not np.array_equal(lv.part_keys, x[order]):
            fails.append(f"{tag}: partition differs from the stable closed form")
    return fails


def pin_scaled_closed_form(O, lib) -> list[str]:
    """x_k = x_min + k w (w a power of two), beta = 2(n-1): the scale is
    exactly 2/w, so i(x_k) = 2k and b_i = floor(i/2) + 1 for the full sample."""
    fails = []
    rng = np.random.default_rng(3)
    for n, lo, w in ((500, -3.0, 0.25), (1024, 1e6, 2.0 ** -10), (300, -(2.0 ** 40), 2.0 ** 30)):
        k = rng.permutation(n)
        x = lo + k.astype(np.float64) * w
        beta = 2 * (n - 1)
        gamma = 50
        lv = O.level(x, n, beta, gamma, 0, sample_idx=np.arange(n, dtype=np.uint64), lib=lib)
        i = np.arange(beta + 1, dtype=np.int64)
        want_b = i // 2 + 1
        if not np.array_equal(lv.b.astype(np.int64), want_b):
            fails.append(f"n={n} lo={lo} w={w}: b differs from floor(i/2) + 1")
        if lv.scale != 2.0 / w:
            fails.append(f"n={n}: scale {lv.scale} != 2/w")
    return fails


def lfail_bound(n, alpha, beta, gamma, delta, ratio=1.0):
    """Right side of the bucketing-failure lemma (Sec. 3.3), or None if K < 1."""
    K = gamma * delta / (2.0 * n) - 2.0 * ratio * gamma / beta
    if K < 1.0:
        return None
    return (2.0 * n / delta) * math.exp(-(alpha * K / (2.0 * gamma)) * (1.0 - 1.0 / K) ** 2)


def pin_lfail(O, lib) -> list[str]:
    """Empirical frequency of a bucket larger than delta (Sec. 4.2 protocol) on
    uniform keys (sigma2/sigma1 = 1) must respect the lemma's bound; the same
    holds for a sorted array because the samples are uniform draws.  A
    one-sample model must fail every time (the check is not vacuous)."""
    fails = []
    n = 100_000
    x = datagen.f64("uniform", n, 21)
    xs = np.sort(x)
    r = O.root34(n, lib=lib)
    reps = 8
    for name, arr, (a, be, g, d) in [
        ("paper params", x, (r, r, r, r)),
        ("paper params, sorted input", xs, (r, r, r, r)),
        ("b=0.85", x, (r, int(n ** 0.85), r, r)),
    ]:
        bound = lfail_bound(n, a, be, g, d)
        fcount = 0
        for rep in range(reps):
            lv = O.level(arr, a, be, g, O.node_seed(1000 + rep, 0, 0, 0, lib=lib), lib=lib)
            if lv.sizes.max() > d:
                fcount += 1
        if bound is None or bound > 1e-6:
            fails.append(f"{name}: test setup expects a tiny bound, got {bound}")
        elif fcount:
            fails.append(f"{name}: {fcount}/{reps} bucketing failures, bound {bound:.3g}")
    # control: a single sample leaves at most two non-empty buckets
    fcount = 0
    for rep in range(4):
        lv = O.level(x, 1, r, r, O.node_seed(2000 + rep, 0, 0, 0, lib=lib), lib=lib)
        fcount += int(lv.sizes.max() > r)
    if fcount != 4:
        fails.append(f"control: one-sample model failed only {fcount}/4 times")
    return fails


def depth_bound(n, tau):
    """Depth limit from the worst-case lemma (Sec. 3.2): a bucket that recurses
    at depth i holds fewer than n^{(3/4)^i} keys, and arrays below tau stop."""
    return math.ceil(math.log(math.log(n) / math.log(tau), 4.0 / 3.0)) + 1


def pin_depth(O, lib) -> list[str]:
    """Recursion depth stays within the lemma's bound, also on an input built to
    defeat equal-width bins (x_i = 2^-i puts almost everything in bin 0)."""
    fails = []
    adversarial = np.array([2.0 ** (-i) for i in range(1000)])
    for name, x in [("uniform 1e6", datagen.config1()),
                    ("lognormal 2e5", datagen.f64("lognormal", 200_000, 9)),
                    ("geometric 1000", adversarial)]:
        s, _, st = O.sort(x, lib=lib)
        lim = depth_bound(x.shape[0], 100)
        if st["max_depth"] > lim:
            fails.append(f"{name}: depth {st['max_depth']} > bound {lim}")
        if not np.array_equal(s, np.sort(x)):
            fails.append(f"{name}: not sorted")
    return fails


# ---- Spline Learned Sort (App. A.5) -------------------------------------------

def _bucket_of(lv, x):
    """Bucket index of every (distinct) key of x, read off the partition."""
    sizes = lv.sizes.astype(np.int64)
    owner = np.repeat(np.arange(sizes.shape[0]), sizes)
    where = {float(k) if x.dtype == np.float64 else int(k): int(j)
             for k, j in zip(lv.part_keys, owner)}
    return np.array([where[float(k) if x.dtype == np.float64 else int(k)] for k in x])


def _grid_keys(beta, extra, rng):
    """Keys on [0, beta] with x_min = 0 and x_max = beta, so the scale is
    exactly 1 and a key's position in bin units is the key itself."""
    mids = np.arange(beta, dtype=np.float64) + 0.5
    ints = np.arange(beta + 1, dtype=np.float64)
    more = np.unique(np.floor(rng.random(extra) * beta * 1024.0) / 1024.0 + 1.0 / 2048.0)
    x = np.unique(np.concatenate([mids, ints, more]))
    return rng.permutation(x)


def pin_spline_library_sort(O, lib) -> list[str]:
    """Spline Learned Sort sorts: numpy's order, stable payload, brute force."""
    fails = []
    cases = [(d, datagen.f64(d, 20_000, 300 + i)) for i, d in enumerate(datagen.F64_DISTS)]
    cases += [(k, datagen.u64(k, 20_000, 400 + i, distinct=300))
              for i, k in enumerate(datagen.U64_KINDS)]
    cases.append(("dup_f64", np.round(datagen.f64("normal", 30_000, 8), 2) + 0.0))
    for name, x in cases:
        s, idx, _ = O.argsort(x, lib=lib, model="spline")
        if not np.array_equal(s, np.sort(x, kind="stable")):
            fails.append(f"spline {name}: keys differ from numpy sort")
        if not np.array_equal(idx, _np_stable_argsort(x)):
            fails.append(f"spline {name}: argsort differs from numpy stable argsort")
    base = [1.0, 1.0, 2.0, 2.5, 3.0, 7.0]
    for perm in itertools.permutations(range(len(base))):
        x = np.array([base[q] for q in perm], dtype=np.float64)
        s, idx, _ = O.argsort(x, tau=2, lib=lib, model="spline")
        want = sorted(range(len(x)), key=lambda i: (x[i], i))
        if list(idx) != want:
            fails.append(f"spline permutation {perm}: got {list(idx)} want {want}")
            break
    return fails


def pin_spline_identity(O, lib) -> list[str]:
    """One sample per bin (b_i = i + 1): the spline is then the identity in bin
    units, F(x) alpha = x, so every key's bucket is floor(x gamma / alpha); a
    dropped interpolation term or the wrong end of the bin breaks it."""
    fails = []
    rng = np.random.default_rng(31)
    for beta, gamma in ((64, 63), (500, 37), (1000, 1000)):
        x = _grid_keys(beta, 3000, rng)
        pos = {float(v): i for i, v in enumerate(x)}
        sidx = np.array([pos[j + 0.5] for j in range(beta)] + [pos[float(beta)]], dtype=np.uint64)
        alpha = beta + 1
        lv = O.level(x, alpha, beta, gamma, 0, sample_idx=sidx, lib=lib, model="spline")
        if not np.array_equal(lv.b.astype(np.int64), np.arange(1, beta + 2)):
            fails.append(f"beta={beta}: b differs from i + 1")
            continue
        want = np.floor((x * float(gamma)) / float(alpha)).astype(np.int64)
        got = _bucket_of(lv, x)
        if not np.array_equal(got, want):
            bad = int(np.sum(got != want))
            fails.append(f"beta={beta} gamma={gamma}: {bad} keys off the closed form")
    return fails


def pin_spline_thresholds(O, lib) -> list[str]:
    """The spline interpolates the PCF's values at the bin thresholds: a key on
    the threshold t_k (position exactly k) takes the PCF bucket of bin k - 1,
    and no key of bin k leaves the PCF range [T_{k-1}, T_k] (same samples)."""
    fails = []
    rng = np.random.default_rng(32)
    for beta, gamma, alpha in ((256, 100, 300), (1000, 400, 700)):
        x = _grid_keys(beta, 5000, rng)
        ns = O.node_seed(5, 0, 0, 0, lib=lib)
        sp = O.level(x, alpha, beta, gamma, ns, lib=lib, model="spline")
        pc = O.level(x, alpha, beta, gamma, ns, lib=lib, model="pcf")
        if not np.array_equal(sp.b, pc.b):
            fails.append(f"beta={beta}: the two models trained differently")
            continue
        T = pc.T.astype(np.int64)
        got = _bucket_of(sp, x)
        k = np.minimum(np.floor(x).astype(np.int64), beta)
        on = x == np.floor(x)
        want_on = np.where(k == 0, 0, T[np.maximum(k - 1, 0)])
        if not np.array_equal(got[on], want_on[on]):
            fails.append(f"beta={beta}: threshold keys off the PCF value of the previous bin")
        lo = np.where(k == 0, 0, T[np.maximum(k - 1, 0)])
        if np.any(got < lo) or np.any(got > T[k]):
            fails.append(f"beta={beta}: a key left its bin's PCF range")
    return fails


def pin_spline_level_invariants(O, lib) -> list[str]:
    fails = []
    rng = np.random.default_rng(33)
    for name, x, (a, be, g) in [
        ("uniform", datagen.f64("uniform", 20_000, 13), (500, 800, 120)),
        ("lognormal", datagen.f64("lognormal", 20_000, 14), (1000, 300, 63)),
        ("dups", np.round(rng.standard_normal(20_000), 1) + 0.0, (700, 700, 700)),
        ("bursty", datagen.u64("bursty", 20_000, 16), (2000, 2000, 100)),
    ]:
        idx = np.arange(x.shape[0], dtype=np.uint32)
        lv = O.level(x, a, be, g, O.node_seed(3, 0, 0, 0, lib=lib), vals=idx, lib=lib,
                     model="spline")
        if lv.status != 0:
            fails.append(f"spline {name}: unexpected status {lv.status}")
            continue
        fails += [f"spline {m}" for m in _check_level(name, x, lv, a, be, g)]
    return fails


def pin_spline_lfail_depth(O, lib) -> list[str]:
    """The spline keeps the PCF's guarantees (App. A.5): no bucket above delta
    on uniform keys with the paper's parameters, and the depth bound."""
    fails = []
    n = 100_000
    x = datagen.f64("uniform", n, 22)
    r = O.root34(n, lib=lib)
    for rep in range(6):
        lv = O.level(x, r, r, r, O.node_seed(3000 + rep, 0, 0, 0, lib=lib), lib=lib,
                     model="spline")
        if lv.sizes.max() > r:
            fails.append(f"spline: bucketing failure on uniform keys (rep {rep})")
    for name, y in [("lognormal 2e5", datagen.f64("lognormal", 200_000, 10)),
                    ("geometric 1000", np.array([2.0 ** (-i) for i in range(1000)]))]:
        s, _, st = O.sort(y, lib=lib, model="spline")
        if st["max_depth"] > depth_bound(y.shape[0], 100):
            fails.append(f"spline {name}: depth {st['max_depth']} over the bound")
        if not np.array_equal(s, np.sort(y)):
            fails.append(f"spline {name}: not sorted")
    return fails


ALL_PINS = [pin_library_sort, pin_brute_force, pin_selection_sort, pin_level_invariants,
            pin_identity_closed_form, pin_scaled_closed_form, pin_halved_range_closed_form, pin_lfail, pin_depth,
            pin_spline_library_sort, pin_spline_identity, pin_spline_thresholds,
            pin_spline_level_invariants, pin_spline_lfail_depth]
