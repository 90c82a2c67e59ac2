"""Host model of the GPU's standard sort for failed buckets (radix levels).

The HIP library sorts a bucket that failed (|c_j| >= delta, Algorithm 1) and
does not fit LDS with radix levels over order-preserving 64-bit key images.
Each radix node has 256 buckets.  Its digit is linear (the 8 bits below the
top of its range) unless 256 samples show most keys in the lowest linear
digit spread over eight or more octaves; then the digit is logarithmic (the
octave and the two bits after the leading one).  A linear digit removes 8
bits of range per level, a log digit only 3, and a call runs a bounded number
of levels.  This model replays that rule level by level on the host so the
level count an input needs can be compared with what a call has.

It models the library's rule, not the paper's algorithm, and shares no code
with the library: sample positions come from numpy's generator, so only the
structure of the decision is reproduced.
"""
from __future__ import annotations

import numpy as np

RS = 256       # samples that choose a radix node's digit scale
NBITS = 8      # bits of a linear digit (256 buckets)
_POW2 = np.array([1 << k for k in range(64)], dtype=np.uint64)


def bitlen(v: np.ndarray) -> np.ndarray:
    """Number of significant bits of each uint64 (0 for 0)."""
    return np.searchsorted(_POW2, np.asarray(v, dtype=np.uint64), side="right").astype(np.int64)


def images_f64(x: np.ndarray) -> np.ndarray:
    """Order-preserving uint64 images of finite fp64 keys."""
    b = x.view(np.uint64)
    neg = (b >> np.uint64(63)) == 1
    return np.where(neg, ~b, b | np.uint64(1 << 63))


def root34(n: int) -> int:
    m = int(round(n ** 0.75))
    while m ** 4 > n ** 3:
        m -= 1
    while (m + 1) ** 4 <= n ** 3:
        m += 1
    return m


def chain_levels(n: int, cap: int = 8192) -> int:
    """Levels of a call's fixed chain: the delta rule's model levels for n keys
    plus the radix levels of a 64-bit range (8 linear levels and the level that
    marks single-valued nodes done)."""
    d, m = 0, n
    while m > cap:
        m = root34(m)
        d += 1
    return d + 9


def _log_digit(off: np.ndarray) -> np.ndarray:
    e = bitlen(off)
    sh = np.maximum(e - 3, 0).astype(np.uint64)
    mant = ((off >> sh) & np.uint64(3)).astype(np.int64)
    return np.where(e <= 2, off.astype(np.int64), (e - 2) * 4 + mant)


def deepest_level(nodes: list[np.ndarray], start_level: int, nlev: int, budgeted: bool,
                  seed: int = 0, cap: int = 8192) -> int:
    """Runs the radix levels from `start_level` over `nodes` (arrays of key
    images, each a radix node) and returns the deepest level that holds a
    node.  budgeted=False: log digits whenever the samples ask for them;
    budgeted=True: only while the levels after this one (of nlev in all) can
    still finish a child of the node's range minus 3 bits with linear digits."""
    rng = np.random.default_rng(seed)
    level = start_level
    live = [x for x in nodes if x.shape[0] > cap]
    deepest = start_level - 1
    while live:
        deepest = level
        nxt = []
        for x in live:
            lo, hi = x.min(), x.max()
            if lo == hi:
                continue  # single-valued: marked done on this level
            bl = int(bitlen(np.array([hi - lo]))[0])
            shift = max(0, bl - NBITS)
            left = nlev - level - 1
            log_ok = (not budgeted) or ((bl - 3 + 7) // 8 + 1 <= left)
            logd = False
            off = x - lo
            if bl - 1 >= 16 and x.shape[0] >= RS and log_ok:
                s = off[rng.integers(0, x.shape[0], RS)]
                dg = (s >> np.uint64(shift)).astype(np.int64)
                cnt = np.bincount(dg)
                best = int(np.argmax(cnt))
                c = int(cnt[best])
                if c >= RS // 2:
                    sel = np.sort(s[dg == best])
                    e0 = int(bitlen(sel[c // 10:c // 10 + 1])[0])
                    e1 = int(bitlen(sel[c - 1 - c // 10:c - c // 10])[0])
                    logd = e1 >= e0 + 8
            digit = _log_digit(off) if logd else (off >> np.uint64(shift)).astype(np.int64)
            order = np.argsort(digit, kind="stable")
            d_sorted = digit[order]
            cuts = np.flatnonzero(np.diff(d_sorted)) + 1
            for part in np.split(order, cuts):
                if part.shape[0] > cap:
                    nxt.append(x[part])
        live = nxt
        level += 1
    return deepest
