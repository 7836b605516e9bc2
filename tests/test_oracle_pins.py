"""The CPU oracle against facts fixed by the paper and by mathematics."""
import pytest

from oracle.oracle import OracleLib
from tests import pins


@pytest.fixture(scope="module")
def O():
    return OracleLib()


@pytest.mark.parametrize("pin", pins.PINS, ids=lambda f: f.__name__)
def test_pin(O, pin):
    pin(O)
