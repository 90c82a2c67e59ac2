"""Level budget of the standard sort for failed buckets (host model, no GPU).

Algorithm 1's standard-sort fallback always finishes, so a call must never
run out of levels.  A call's fixed chain has the delta rule's levels plus 9
(8 linear radix levels of 8 bits and one level that marks single-valued
nodes done).  Log-scale radix digits remove only 3 bits per level; keys in
nested shells of widely different scales ask for them on every level.  The
model of tests/radix_levels_model.py shows that such an input needs more
levels than the chain of a 2^27-key call holds when log digits are taken
freely, and fits when they are taken only while the levels left can still
finish a node's children linearly (the rule the library's fit kernel uses).

The model runs at 2^22 keys with an LDS capacity of 256 keys: the level count
depends on the ratio of keys to capacity, which is the same as for 2^27 keys
and the library's 8192."""
import numpy as np

from paper_2405_07122_amd import datagen
from tests import radix_levels_model as M


def _shell_node(n, seed):
    x = datagen.nested_scales(n, seed)
    # the root's model (level 0) puts every shell key into its first bin, far
    # below the outliers at 1.0: one failed bucket, a radix node on level 1
    return M.images_f64(x[x < 0.5])


def test_nested_scales_exhaust_the_chain_without_the_budget():
    nlev = M.chain_levels(2 ** 27)
    assert nlev == 12
    node = _shell_node(2 ** 22, 5)
    free = [M.deepest_level([node], 1, nlev, budgeted=False, seed=s, cap=256) for s in (0, 2)]
    budgeted = [M.deepest_level([node], 1, nlev, budgeted=True, seed=s, cap=256) for s in (0, 2)]
    # levels 0 .. nlev - 1 exist: a node on level >= nlev is never sorted
    assert max(free) >= nlev, free
    assert max(budgeted) <= nlev - 1, budgeted


def test_budget_rule_keeps_every_radix_node_finishable():
    """Invariant behind the rule: a radix node of bl bits on level L has
    ceil(bl / 8) + 1 <= nlev - L.  It holds for a node made on level L <= nlev - 9
    (bl <= 64), and each level keeps it: a linear child loses 8 bits, a log
    child 3 bits and is allowed only when ceil((bl - 3) / 8) + 1 <= nlev - L - 1."""
    for nlev in range(9, 16):
        for L0 in range(0, nlev - 8):
            for bl0 in range(1, 65):
                # walk the worst case: log digits whenever allowed (3 bits), else linear
                L, bl = L0, bl0
                assert (bl + 7) // 8 + 1 <= nlev - L
                while bl > 0:
                    left = nlev - L - 1
                    if bl - 1 >= 16 and (bl - 3 + 7) // 8 + 1 <= left:
                        bl -= 3
                    else:
                        bl = max(0, bl - 8)
                    L += 1
                    assert (bl + 7) // 8 + 1 <= nlev - L, (nlev, L0, bl0, L, bl)
                # the single-valued children are marked done on level L <= nlev - 1
                assert L <= nlev - 1
