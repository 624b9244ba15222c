"""The CPU oracle against the pins of tests/pins.py (closed forms, a worked
example, exact brute force, invariants)."""
import pytest

import oracle
import pins


@pytest.mark.parametrize("pin", pins.ALL_PINS, ids=lambda p: p.__name__)
def test_pin(pin):
    fails = pin(oracle.chi0_oracle)
    assert not fails, fails
