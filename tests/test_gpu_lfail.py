"""The bucketing-failure experiment (Sec. 4.2, Fig. 3) on the GPU against the
oracle: with the same node seeds every (cell, array) run is one oracle level,
so the failure counts must agree exactly; and on uniform keys the counts
respect the lemma of Sec. 3.3 where its bound is small."""
import numpy as np
import pytest

from paper_2405_07122_amd import datagen
from tests.gpu_util import banner

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def P():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2405_07122_amd import pcfsort
    pcfsort.load()
    return pcfsort


def test_lfail_counts_match_oracle(P, oracle):
    import torch
    banner("lfail grid vs oracle")
    n, reps, seed = 20_000, 6, 77
    arrays = np.stack([datagen.f64("uniform", n, 900 + r) for r in range(reps)])
    cells = []
    for a, b, c, d in [(0.75, 0.75, 0.75, 0.75), (0.3, 0.75, 0.75, 0.75), (0.75, 0.2, 0.75, 0.6),
                       (0.5, 0.9, 0.9, 0.7), (0.9, 0.5, 0.3, 0.5), (0.2, 0.95, 0.6, 0.75),
                       (0.05, 0.05, 0.05, 0.05), (0.95, 0.95, 0.95, 0.95)]:
        cells.append(tuple(max(1, int(np.floor(n ** v))) for v in (a, b, c, d)))
    got = P.pcf_lfail_grid(torch.from_numpy(arrays).to("cuda"), cells, seed=seed)
    want = np.zeros(len(cells), dtype=np.uint32)
    for ci, (al, be, ga, de) in enumerate(cells):
        for r in range(reps):
            lv = oracle.level(arrays[r], al, be, ga, oracle.node_seed(seed, ci, r, 0))
            want[ci] += int(lv.sizes.max() > de)
    np.testing.assert_array_equal(got, want)
    assert want.min() < reps and want.max() > 0  # both outcomes occur


def test_lfail_bound_holds_at_paper_size(P):
    import torch
    banner("lfail n=1e6 row")
    from tests.oracle_pins import lfail_bound
    n, reps = 1_000_000, 10
    arrays = torch.from_numpy(np.stack([datagen.f64("uniform", n, 950 + r) for r in range(reps)]))
    cells, bounds = [], []
    for a in np.arange(0.05, 0.951, 0.05):
        al, be, ga, de = (max(1, int(np.floor(n ** v))) for v in (a, 0.75, 0.75, 0.75))
        cells.append((al, be, ga, de))
        bounds.append(lfail_bound(n, al, be, ga, de))
    got = P.pcf_lfail_grid(arrays.to("cuda"), cells, seed=5)
    for (cell, bd, f) in zip(cells, bounds, got):
        if bd is not None and bd < 0.05:
            assert f == 0, (cell, bd, f)
    assert got[0] == reps  # one or two samples: buckets are far too coarse
