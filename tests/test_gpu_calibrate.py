"""The roofline's instruction-rate measurement runs and returns plausible
rates (it is a measurement helper, not part of the method)."""
import pytest

from tests.conftest import load_binding

pytestmark = pytest.mark.gpu
B = load_binding()


def test_valu_rates():
    rates = B.ising_valu_rates()
    assert set(rates) == set(B.VALU_RATE_NAMES)
    full = 256 * 64 * 2.4e9  # lane-operations/s at the full VALU rate
    for name, r in rates.items():
        assert 0.05 * full < r < 1.2 * full, (name, r)


def test_lds_rate():
    """LDS read bandwidth: above a tenth of 128 bytes per clock per CU and
    below four times it."""
    r = B.ising_lds_rate()
    ref = 256 * 128 * 2.4e9
    assert 0.1 * ref < r < 4 * ref, r
