"""Seeded input generators (CPU): reproducible, inside their stated bounds."""
import numpy as np

from synth import curved_fault, ensemble_sizes, smooth_slip_rate, straight_fault


def test_ensemble_sizes_are_seeded_and_bounded():
    a = ensemble_sizes(64, 1024, 16384, 5)
    b = ensemble_sizes(64, 1024, 16384, 5)
    assert np.array_equal(a, b)
    assert a.min() >= 1024 and a.max() <= 16384 and len(a) == 64
    # log-uniform: about half of the draws lie below the geometric midpoint 4096
    assert 20 <= int((a < 4096).sum()) <= 44


def test_smooth_slip_rate_is_standardized():
    d = smooth_slip_rate(300, 200, 20, 40, 3)
    assert abs(d.mean()) < 1e-12 and abs(d.std() - 1.0) < 1e-12


def test_fault_elements_have_unit_length():
    for xa, xb in (straight_fault(50), curved_fault(200)):
        assert np.allclose(np.hypot(*(xb - xa).T), 1.0, atol=1e-9)
        assert np.allclose(xa[1:], xb[:-1])
