"""The FP64 oracle against its pins (closed forms, invariants, brute force)."""
import pytest

from tests import oracle_pins

PINS = oracle_pins.ALL_PINS


@pytest.mark.parametrize("pin", PINS, ids=[p.__name__ for p in PINS])
def test_oracle_pin(orc, pin):
    pin(orc)
