"""The oracle's acceptance measures against their pins (measure_pins.py)."""
import pytest

import measure_pins
from oracle import oracle as _oracle_mod


@pytest.mark.parametrize("pin", measure_pins.ALL_PINS, ids=lambda f: f.__name__)
def test_measure_pin(pin):
    pin(_oracle_mod)
