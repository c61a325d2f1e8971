"""The CPU oracle against facts the paper and mathematics fix (no GPU)."""
import pytest

import oracle_pins as P

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


@pytest.mark.parametrize("pin", P.ALL_PINS, ids=lambda p: p.__name__)
def test_pin(orc, pin):
    pin(orc)
