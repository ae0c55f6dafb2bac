"""The CPU oracle against the paper's worked examples, field and S-box
invariants, the OpenSSL command-line tool and structural properties."""
import pytest

from tests import pins


@pytest.mark.parametrize("pin", pins.ALL_PINS, ids=lambda p: p.__name__)
def test_pin(oracle_lib, pin):
    if pin in pins.OPENSSL_PINS and not pins.openssl_available():
        pytest.skip("openssl command-line tool not installed")
    pin(oracle_lib)
