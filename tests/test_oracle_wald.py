"""Pins of the Wald-test oracle (oracle/wald.py) against facts of the normal
distribution that do not depend on its code."""
import math

import numpy as np
import pytest
from scipy import integrate, stats

from oracle.wald import wald


@pytest.mark.parametrize("z,p", [(0.0, 1.0), (1.6448536269514722, 0.10), (1.959963984540054, 0.05),
                                 (2.5758293035489004, 0.01), (3.2905267314919255, 0.001),
                                 (5.326723886384500, 1e-7)])
def test_textbook_two_sided_quantiles(z, p):
    for sign in (1.0, -1.0):
        zz, pp = wald(sign * z * 0.37, 0.37)
        assert abs(zz - sign * z) < 1e-15 * max(1.0, z)
        assert abs(pp - p) < 1e-12 * p


def test_normal_and_chi_square_tails():
    z = np.concatenate([np.linspace(-8, 8, 161), [12.0, -20.0, 30.0]])
    _, p = wald(z, np.ones_like(z))
    assert np.allclose(p, 2.0 * stats.norm.sf(np.abs(z)), rtol=1e-12, atol=0)
    assert np.allclose(p, stats.chi2.sf(z * z, 1), rtol=1e-10, atol=0)


def test_numerical_integration_of_the_density():
    phi = lambda x: math.exp(-0.5 * x * x) / math.sqrt(2.0 * math.pi)
    for z in (0.3, 1.1, 2.7, 4.4):
        tail, err = integrate.quad(phi, z, np.inf, epsabs=0, epsrel=1e-13)
        _, p = wald(z, 1.0)
        assert abs(p - 2.0 * tail) < 1e-11 * p


def test_asymptotic_tail_series():
    """Far tail: P(|Z| > z) = 2 phi(z) / z (1 - 1/z^2 + 3/z^4 - 15/z^6 + ...)."""
    for z in (25.0, 30.0, 37.0):
        phi = math.exp(-0.5 * z * z) / math.sqrt(2.0 * math.pi)
        series = 2.0 * phi / z * (1 - 1 / z**2 + 3 / z**4 - 15 / z**6 + 105 / z**8)
        _, p = wald(-z * 2.0, 2.0)
        assert abs(p - series) < 1e-10 * series


def test_monotone_symmetric_and_nan():
    z = np.linspace(0, 10, 1001)
    _, p = wald(z, 1.0)
    assert np.all(np.diff(p) < 0)
    _, pm = wald(-z, 1.0)
    assert np.array_equal(p, pm)
    zz, pn = wald(np.array([np.nan, 1.0]), np.array([1.0, np.nan]))
    assert np.isnan(zz).all() and np.isnan(pn).all()
