"""Host logic of the critical-Grashof iteration (no GPU): the choice of the
leading eigenvalue and the check of the adjoint slope against the secant."""
import numpy as np

from paper_1905_11601_amd.drivers import gr_slope, leading_index


def test_leading_index_prefers_largest_real_part_and_positive_imaginary_member():
    lams = np.array([-0.1 + 2.0j, 0.3 - 1.5j, 0.3 + 1.5j, 0.2 + 0.0j])
    assert leading_index(lams) == 2
    assert leading_index(np.array([0.1 + 0.0j, -0.2 + 0.0j])) == 0
    # a conjugate pair whose real parts differ by rounding only
    assert leading_index(np.array([0.25 - 1j, 0.25 + 1e-16 + 1j])) == 1


def test_gr_slope_keeps_a_consistent_adjoint_estimate():
    last = (1.0e6, -0.01 + 1.5j)
    lam = -0.005 + 1.5001j
    sec = (lam.real - last[1].real) / (1.1e6 - 1.0e6)
    slope, how = gr_slope(1.5 * sec + 0.3j, 1.1e6, lam, last)
    assert how == "adjoint" and slope == 1.5 * sec
    slope, how = gr_slope(2e-7, 1e6, lam, None)        # first iterate: no secant
    assert how == "adjoint" and slope == 2e-7


def test_gr_slope_falls_back_to_the_secant():
    last = (1.0e6, -0.01 + 1.5j)
    lam = -0.005 + 1.5001j
    sec = (lam.real - last[1].real) / (1.1e6 - 1.0e6)
    assert gr_slope(-sec, 1.1e6, lam, last) == (sec, "secant")        # wrong sign
    assert gr_slope(10 * sec, 1.1e6, lam, last) == (sec, "secant")    # 10x off
    # a different mode led the previous iterate: no secant through it
    slope, how = gr_slope(-sec, 1.1e6, lam, (1.0e6, -0.01 + 2.0j))
    assert how == "adjoint" and slope == -sec
