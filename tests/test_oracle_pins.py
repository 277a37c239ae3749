"""The oracle against the closed forms, exact cases, invariants and library
routines that pin it (see oracle_pins.py for what each pin fixes)."""
import pytest

import oracle_pins


@pytest.mark.parametrize("pin", oracle_pins.ALL_PINS, ids=lambda f: f.__name__)
def test_pin(pin, oracle_lib):
    pin(oracle_lib)
