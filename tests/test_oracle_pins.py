"""The CPU oracle against its pins (brute force, closed forms, invariants, the
worked example of Section 2.2)."""
import pytest

from tests import pins_oracle


@pytest.mark.parametrize("pin", pins_oracle.ALL_PINS, ids=lambda f: f.__name__)
def test_oracle_pin(pin, oracle_lib):
    pin(oracle_lib)
