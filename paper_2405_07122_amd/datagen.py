"""Seeded synthetic inputs shaped like the paper's workloads.

This module holds no sorting arithmetic: it only draws keys.  Both the CPU
oracle (through the tests) and the HIP library consume the arrays it returns,
so the two sides always sort the same bytes.

Distributions (Sec. 4, setup paragraph): Uniform(0, 1), Normal(0, 1),
Exponential(1), LogNormal(0, 1); chi-squared(4) and an
8-Gaussian mixture are added.  The paper's real datasets (App. B) are not available;
three uint64 generators stand in for their shapes: heavy duplicates (Zipf),
clustered identifiers and bursty timestamps.  Every fp64 key is finite and
canonicalised with ``x + 0.0`` so that -0.0 never occurs.
"""
from __future__ import annotations

import numpy as np

F64_DISTS = ("uniform", "normal", "lognormal", "exponential", "chi2_4", "mix8")
U64_KINDS = ("zipf", "clustered", "bursty")

# seeds of the single-array throughput workloads (one per distribution)
F64_SEEDS = {"uniform": 1, "normal": 2, "lognormal": 3, "exponential": 4, "chi2_4": 5, "mix8": 6}
U64_SEEDS = {"zipf": 7, "clustered": 8, "bursty": 9}

_CHUNK = 1 << 24


def _canon(x: np.ndarray) -> np.ndarray:
    x += 0.0  # maps -0.0 to +0.0 under round-to-nearest
    return x


def f64(dist: str, n: int, seed: int) -> np.ndarray:
    """n i.i.d. fp64 keys of distribution `dist` from `seed`."""
    rng = np.random.default_rng(seed)
    out = np.empty(n, dtype=np.float64)
    if dist == "mix8":
        # component parameters are drawn first from the same stream
        means = rng.uniform(-100.0, 100.0, size=8)
        sigmas = rng.uniform(0.1, 5.0, size=8)
    for a in range(0, n, _CHUNK):
        m = min(_CHUNK, n - a)
        if dist == "uniform":
            out[a:a + m] = rng.random(m)
        elif dist == "normal":
            out[a:a + m] = rng.standard_normal(m)
        elif dist == "lognormal":
            out[a:a + m] = np.exp(rng.standard_normal(m))
        elif dist == "exponential":
            out[a:a + m] = rng.standard_exponential(m)
        elif dist == "chi2_4":
            out[a:a + m] = rng.chisquare(4.0, m)
        elif dist == "mix8":
            comp = rng.integers(0, 8, size=m)
            out[a:a + m] = means[comp] + sigmas[comp] * rng.standard_normal(m)
        else:
            raise ValueError(f"unknown distribution {dist}")
    return _canon(out)


def u64(kind: str, n: int, seed: int, distinct: int = 2_000_000, zipf_s: float = 1.1,
        runs: int = 1000) -> np.ndarray:
    """n uint64 keys of kind zipf | clustered | bursty, shuffled."""
    rng = np.random.default_rng(seed)
    if kind == "zipf":
        # distinct random values, rank k drawn with probability proportional to k^-s
        vals = np.unique(rng.integers(0, np.iinfo(np.uint64).max, size=distinct,
                                      dtype=np.uint64, endpoint=True))
        rng.shuffle(vals)
        w = np.arange(1, vals.shape[0] + 1, dtype=np.float64) ** (-zipf_s)
        cdf = np.cumsum(w)
        cdf /= cdf[-1]
        out = np.empty(n, dtype=np.uint64)
        for a in range(0, n, _CHUNK):
            m = min(_CHUNK, n - a)
            r = np.searchsorted(cdf, rng.random(m), side="right")
            np.minimum(r, vals.shape[0] - 1, out=r)
            out[a:a + m] = vals[r]
        return out
    if kind == "clustered":
        # `runs` increasing runs at log-uniform starts in [1, 2^63), geometric gaps (mean 16)
        out = np.empty(n, dtype=np.uint64)
        per = [n // runs + (1 if r < n % runs else 0) for r in range(runs)]
        starts = np.floor(np.exp2(rng.uniform(0.0, 63.0, size=runs))).astype(np.uint64)
        a = 0
        for r in range(runs):
            m = per[r]
            if m == 0:
                continue
            gaps = rng.geometric(1.0 / 16.0, size=m).astype(np.uint64)
            out[a:a + m] = starts[r] + np.cumsum(gaps, dtype=np.uint64)
            a += m
        rng.shuffle(out)
        return out
    if kind == "bursty":
        # cumulative sum of Pareto(alpha=1.5, x_m=1) increments, floored
        inc = 1.0 + rng.pareto(1.5, size=n)
        t = np.cumsum(inc)
        out = np.floor(t).astype(np.uint64)
        rng.shuffle(out)
        return out
    raise ValueError(f"unknown kind {kind}")


def adversarial(dist: str, n: int, seed: int) -> np.ndarray:
    """The point-mass input of the paper's robustness experiment (App. C): n
    keys of `dist`, plus n copies of one value drawn uniformly inside
    [x_min, x_max] of those keys, shuffled (2n keys in all)."""
    x = f64(dist, n, seed)
    rng = np.random.default_rng(seed + 0x5eed)
    lo, hi = float(x.min()), float(x.max())
    v = lo + rng.random() * (hi - lo)
    v = min(max(v, lo), hi) + 0.0
    out = np.concatenate([x, np.full(n, v, dtype=np.float64)])
    rng.shuffle(out)
    return out


def nested_scales(n: int, seed: int, keep: float = 0.45, top_bits: int = 61,
                  outliers: int = 3) -> np.ndarray:
    """fp64 keys in nested shells of widely different scales (clustered
    identifiers at many magnitudes, packed into tiny positive doubles).

    Keys are built as 64-bit patterns: shell 0 spans offsets [0, 2^b) above the
    smallest normal double with b = top_bits; it holds its minimum, half of a
    fraction 1 - keep of its keys in [2^(b-21), 2^(b-20)) and the other half
    in [2^(b-9), 2^(b-8)), and passes the fraction `keep` on to the next shell,
    which starts at offset 2^(b-1) and has b - 3 bits.  Shells continue while
    b >= 24; the last one is uniform.  `outliers` keys equal to 1.0 stretch the
    value range far beyond the shells.  Shuffled."""
    rng = np.random.default_rng(seed)
    parts = []
    base = np.uint64(1) << np.uint64(52)  # bit pattern of the smallest normal double
    b = top_bits
    m = n - outliers
    while m > 0:
        if b < 24 or m < 64:
            parts.append(base + rng.integers(0, 2 ** b, size=m, dtype=np.uint64))
            break
        inner = int(m * keep)
        rest = m - inner - 1
        lo = rest // 2
        hi = rest - lo
        parts.append(np.array([base], dtype=np.uint64))
        parts.append(base + np.uint64(2 ** (b - 21)) +
                     rng.integers(0, 2 ** (b - 21), size=lo, dtype=np.uint64))
        parts.append(base + np.uint64(2 ** (b - 9)) +
                     rng.integers(0, 2 ** (b - 9), size=hi, dtype=np.uint64))
        base = base + np.uint64(2 ** (b - 1))
        b -= 3
        m = inner
    out = np.concatenate(parts).view(np.float64)
    out = np.concatenate([out, np.ones(outliers, dtype=np.float64)])
    rng.shuffle(out)
    return out


def config1() -> np.ndarray:
    """The plain workload: n = 1e6 fp64 keys, Uniform[0, 1), seed 0."""
    return f64("uniform", 1_000_000, 0)


def config2(dist: str, n: int = 100_000_000) -> np.ndarray:
    """Single-array throughput workload for one distribution (seeds 1-6)."""
    return f64(dist, n, F64_SEEDS[dist])


def config3(kind: str, n: int = 200_000_000) -> np.ndarray:
    """Skewed uint64 workload (seeds 7-9)."""
    return u64(kind, n, U64_SEEDS[kind])


def segments(num: int = 2048, lo_log2: float = 10.0, hi_log2: float = 22.0, seed: int = 10,
             scale: float = 1.0):
    """Batched workload: `num` fp64 segments, sizes floor(2^U[lo, hi]) (times
    `scale`), each drawn from a distribution picked uniformly from F64_DISTS.
    Returns (keys, offsets uint64[num+1], payload uint32 = in-segment index)."""
    rng = np.random.default_rng(seed)
    sizes = np.floor(np.exp2(rng.uniform(lo_log2, hi_log2, size=num)) * scale).astype(np.int64)
    dists = rng.integers(0, len(F64_DISTS), size=num)
    seg_seeds = rng.integers(0, 2**62, size=num)
    offsets = np.zeros(num + 1, dtype=np.uint64)
    offsets[1:] = np.cumsum(sizes)
    total = int(offsets[-1])
    keys = np.empty(total, dtype=np.float64)
    vals = np.empty(total, dtype=np.uint32)
    for s in range(num):
        a, b = int(offsets[s]), int(offsets[s + 1])
        keys[a:b] = f64(F64_DISTS[dists[s]], b - a, int(seg_seeds[s]))
        vals[a:b] = np.arange(b - a, dtype=np.uint32)
    return keys, offsets, vals


def request_trace(rate: float, count: int, seed: int = 11, lo_log2: float = 12.0,
                  hi_log2: float = 26.0):
    """Serving workload: Poisson arrivals at `rate` per second.  Returns a list of
    (arrival_s, n, key_type 'f64'|'u64', distribution) tuples."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate, size=count)
    t = np.cumsum(gaps) - gaps[0]
    sizes = np.floor(np.exp2(rng.uniform(lo_log2, hi_log2, size=count))).astype(np.int64)
    kinds = rng.integers(0, 2, size=count)
    dists = rng.integers(0, len(F64_DISTS), size=count)
    return [(float(t[i]), int(sizes[i]), "f64" if kinds[i] == 0 else "u64",
             F64_DISTS[dists[i]]) for i in range(count)]


def to_u64_request(x: np.ndarray, lo: float) -> np.ndarray:
    """uint64 request keys from an fp64 draw: floor((x - lo) * 2^32), clipped at 0."""
    y = np.maximum(x - lo, 0.0) * 4294967296.0
    return np.floor(y).astype(np.uint64)
