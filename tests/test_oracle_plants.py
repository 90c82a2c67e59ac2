"""Each deliberate mistake compiled into a copy of the oracle must trip a pin.

This shows that the pins in oracle_pins.py are sharp enough to catch the
plausible slips (a dropped term, a wrong operand, an off-by-one, an exclusive
prefix, a broken sampler, a missing fallback, an unstable merge)."""
import os

import pytest

from tests import oracle_pins as P

PLANTS = [
    "PCFO_PLANT_UNSTABLE",
    "PCFO_PLANT_SCALE_OPERAND",
    "PCFO_PLANT_BIN_PLUS_ONE",
    "PCFO_PLANT_EXCLUSIVE_PREFIX",
    "PCFO_PLANT_T_CEIL",
    "PCFO_PLANT_NO_FALLBACK",
    "PCFO_PLANT_SAMPLE_PREFIX",
    "PCFO_PLANT_SPLINE_UPPER",
    "PCFO_PLANT_SPLINE_NOFRAC",
    "PCFO_PLANT_HALF_OFFSET",
]


@pytest.mark.parametrize("plant", PLANTS)
def test_plant_is_caught(oracle, plant, tmp_path):
    path = str(tmp_path / f"liboracle_{plant}.so")
    oracle.build(path, extra_flags=[f"-D{plant}"])
    lib = oracle.load(path)
    caught = []
    for pin in P.ALL_PINS:
        try:
            fails = pin(oracle, lib)
        except RecursionError:
            fails = ["recursion overflow"]
        except Exception as e:  # an exception inside a pin is also a catch
            fails = [repr(e)]
        if fails:
            caught.append(pin.__name__)
    assert caught, f"{plant} was not caught by any pin"
