"""Pins for the prior transforms (Table 1 of the paper): CDF round trips and
closed-form moments of each prior shape, plus the periodic-coordinate set."""
import math

import numpy as np
import pytest

import oracle
from paper_2509_04336_amd import inputs


@pytest.fixture(scope="module")
def ev11():
    spec = inputs.paper_event(with_noise=False)
    return oracle.event_from_spec(spec)


def _theta_of(ev, j, u):
    uu = np.full(ev.ndim, 0.5)
    uu[j] = u
    return oracle.prior_transform(ev, uu)[j]


def test_uniform_cdf_roundtrip(ev11):
    lo, hi = inputs.PRIOR_PAPER_LO, inputs.PRIOR_PAPER_HI
    for j in (0, 1, 2, 3, 6, 8, 9, 10):
        for u in np.linspace(0, 1, 17):
            x = _theta_of(ev11, j, u)
            assert abs((x - lo[j]) / (hi[j] - lo[j]) - u) < 1e-12


def test_powerlaw2_cdf_roundtrip_and_mean(ev11):
    a, b = 100.0, 5000.0
    for u in np.linspace(0, 1, 33):
        x = _theta_of(ev11, 4, u)
        assert abs((x**3 - a**3) / (b**3 - a**3) - u) < 1e-12
    # E[dL] for p ~ x^2 on [a, b] is 3/4 (b^4 - a^4) / (b^3 - a^3); midpoint rule
    # over a fine u grid integrates the inverse CDF.
    n = 20000
    us = (np.arange(n) + 0.5) / n
    xs = np.array([_theta_of(ev11, 4, u) for u in us])
    mean = xs.mean()
    exact = 0.75 * (b**4 - a**4) / (b**3 - a**3)
    assert abs(mean - exact) / exact < 1e-5


def test_sine_prior(ev11):
    for u in np.linspace(0, 1, 33):
        x = _theta_of(ev11, 5, u)
        assert abs((1.0 - math.cos(x)) / 2.0 - u) < 1e-12
    us = (np.arange(4000) + 0.5) / 4000
    xs = np.array([_theta_of(ev11, 5, u) for u in us])
    assert abs(np.mean(np.cos(xs) ** 2) - 1.0 / 3.0) < 1e-6
    assert abs(np.mean(xs) - math.pi / 2) < 1e-9


def test_cosine_prior(ev11):
    for u in np.linspace(0, 1, 33):
        x = _theta_of(ev11, 7, u)
        assert abs((math.sin(x) + 1.0) / 2.0 - u) < 1e-12
    us = (np.arange(4000) + 0.5) / 4000
    xs = np.array([_theta_of(ev11, 7, u) for u in us])
    assert abs(np.mean(np.sin(xs) ** 2) - 1.0 / 3.0) < 1e-6
    assert abs(np.mean(xs)) < 1e-9


def test_fixed_parameters_for_4d():
    spec = inputs.tiny_event()
    ev = oracle.event_from_spec(spec)
    th = oracle.prior_transform(ev, [0.0, 1.0, 0.5, 0.25])
    assert th[0] == 20.0 and th[1] == 1.0 and th[2] == 0.0 and abs(th[3] + 0.45) < 1e-15
    assert np.array_equal(th[4:], spec.fixed_theta[4:])


def test_periodic_set():
    lib = oracle.lib()
    assert [j for j in range(11) if lib.or_is_periodic(11, j)] == [6, 8, 9]
    assert not any(lib.or_is_periodic(4, j) for j in range(4))
