"""Pins of the oracle's diagnostics (CPU only): volume fraction, its threshold
variant and mass, against hand counts and closed forms that do not use the
oracle's own h(eta).

The volume fraction is the mean of H = sum_v h(eta_v) with the interpolation
function h(eta) = eta^3 (6 eta^2 - 15 eta + 10) of the model formulation
(Methods, "Phase-field model formulation"); the threshold variant counts the
points whose largest order parameter exceeds 1/2.
"""
import numpy as np
import pytest

from oracle import diagnostics as dg
from oracle import model as om
from oracle import spectral as sp


def _state(c, eta):
    return om.to_kspace(c, eta)


def test_uniform_order_parameter_gives_h_of_it(params):
    """eta_1 = a everywhere: vf = h(a), worked by hand; c does not enter."""
    shape = (8, 10, 12)
    m = om.Model(shape, params)
    rng = np.random.default_rng(4)
    for a, h_a, thr in ((0.3, 0.16308, 0.0), (0.7, 0.83692, 1.0)):
        # h(0.3) = 0.027 (0.54 - 4.5 + 10) = 0.16308; h(0.7) = 0.343 (2.94 - 10.5 + 10) = 0.83692
        eta = np.zeros((3,) + shape)
        eta[0] = a
        vfs = []
        for c in (np.full(shape, 0.16), 0.16 + 0.05 * rng.standard_normal(shape)):
            vf, vf_thr = dg.volume_fraction(m, _state(c, eta))
            assert vf == pytest.approx(h_a, rel=1e-13)
            assert vf_thr == thr
            vfs.append(vf)
        assert vfs[0] == vfs[1]


def test_two_level_boxes_hand_count(params):
    """Disjoint boxes on an 8^3 grid: 60 points with eta_1 = 1, 8 points with
    eta_2 = 0.6 and 16 points with eta_3 = 0.4, zero elsewhere.
    vf = (60 + 8 h(0.6) + 16 h(0.4)) / 512 with h(0.6) = 0.216 (2.16 - 9 + 10)
    = 0.68256 and h(0.4) = 0.064 (0.96 - 6 + 10) = 0.31744; the threshold
    variant counts the 60 + 8 points above 1/2."""
    shape = (8, 8, 8)
    m = om.Model(shape, params)
    eta = np.zeros((3,) + shape)
    eta[0, 0:3, 0:4, 0:5] = 1.0            # 60 points
    eta[1, 4:6, 4:6, 4:6] = 0.6            # 8 points
    eta[2, 6:8, 0:2, 4:8] = 0.4            # 16 points
    c = np.full(shape, 0.2)
    vf, vf_thr = dg.volume_fraction(m, _state(c, eta))
    assert vf == pytest.approx((60 + 8 * 0.68256 + 16 * 0.31744) / 512, rel=1e-12)
    assert vf_thr == pytest.approx(68 / 512, abs=1e-15)


def test_smooth_field_closed_form_mean(params):
    """eta_1 = 1/2 + A cos(2 pi x / N + 0.1): h(1/2 + u) is 1/2 plus an odd
    polynomial in u, so the mean is exactly 1/2.  eta_2 = a + b cos(2 pi y / N): a Taylor
    expansion of the quintic about a is exact, odd powers of the cosine average
    to zero on the grid, <cos^2> = 1/2 and <cos^4> = 3/8 (N > 4), so
    <h> = h(a) + h''(a) b^2 / 4 + h''''(a) b^4 / 64, with h'' = 60 e - 180 e^2
    + 120 e^3 and h'''' = 720 e - 360."""
    n = 16
    shape = (n, n, n)
    m = om.Model(shape, params)
    th = 2 * np.pi * np.arange(n) / n
    A, a, b = 0.3, 0.2, 0.1
    eta = np.zeros((3,) + shape)
    eta[0] = (0.5 + A * np.cos(th + 0.1))[None, None, :]
    eta[1] = (a + b * np.cos(th))[None, :, None]
    h_a = a ** 3 * (6 * a * a - 15 * a + 10)
    h2 = 60 * a - 180 * a * a + 120 * a ** 3
    h4 = 720 * a - 360
    expect = 0.5 + h_a + h2 * b * b / 4 + h4 * b ** 4 / 64
    vf, vf_thr = dg.volume_fraction(m, _state(np.full(shape, 0.1), eta))
    assert vf == pytest.approx(expect, rel=1e-13)
    # threshold: eta_1 > 1/2 where cos(2 pi x / 16 + 0.1) > 0, i.e. x in {0..3, 12..15}
    # (the phase keeps every point away from exactly 1/2): 8 of 16 columns
    assert vf_thr == pytest.approx(8 / 16, abs=1e-15)


def test_mass_is_the_mean_of_c(params):
    shape = (8, 6, 10)
    rng = np.random.default_rng(9)
    c = 0.16 + 0.01 * rng.standard_normal(shape)
    y = _state(c, np.zeros((3,) + shape))
    assert dg.mass(y, shape) == pytest.approx(float(np.mean(c)), rel=1e-14)
