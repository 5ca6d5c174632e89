"""Pins for the oracle's TaylorF2 phase and amplitude.

* Low-frequency limit: the phase tends to the Newtonian (0PN) closed form
  (3/128)(pi Mc f)^(-5/3), which depends on the chirp mass only; the first
  correction is O(v^2) (no 0.5PN term).
* Stationary-phase consistency: dPsi/df = 2 pi (t_c - tau(f)) with tau the
  TaylorT2 time to coalescence through 2PN for non-spinning binaries
  (Sathyaprakash & Schutz 2009, Living Rev. Relativ. 12:2).
* Exchange symmetry of the aligned-spin terms (x -> -x, chi_a -> -chi_a).
* Spin-orbit and spin-spin identities: the 1.5PN term equals -16 pi + 4 beta
  and the 2PN spin part equals -10 sigma, with beta and sigma in their
  component-mass form (Poisson & Will 1995; Cutler & Flanagan 1994).
"""
import math

import numpy as np
import pytest

import oracle

TSUN = 1.32712440018e20 / 299792458.0**3


def _theta(mc=30.0, q=0.8, c1=0.0, c2=0.0, tc=0.0, phic=0.0):
    return np.array([mc, q, c1, c2, 1000.0, 0.3, 1.0, 0.2, 0.5, phic, tc])


def _eta(q):
    return q / (1 + q) ** 2


def _Ms(mc, q):
    return mc * _eta(q) ** -0.6 * TSUN


@pytest.mark.parametrize("q", [1.0, 0.8, 0.3])
def test_newtonian_limit_and_q_independence(q):
    mc = 30.0
    th = _theta(mc=mc, q=q)
    devs = []
    for f in (1e-7, 8e-7):
        spa = oracle.phase(th, f) + math.pi / 4
        newton = 3.0 / 128.0 * (math.pi * mc * TSUN * f) ** (-5.0 / 3.0)
        devs.append(spa / newton - 1.0)
        assert abs(devs[-1]) < 1e-4
    # the leading correction scales as v^2 ~ f^(2/3): x8 in f -> x4
    assert abs(devs[1] / devs[0] - 4.0) < 0.02


@pytest.mark.parametrize("q", [1.0, 0.6, 0.25])
def test_stationary_phase_time_relation(q):
    mc, tc = 25.0, 0.013
    th = _theta(mc=mc, q=q, tc=tc)
    eta = _eta(q)
    Ms = _Ms(mc, q)
    for v in (0.02, 0.03):
        f = v**3 / (math.pi * Ms)
        h = f * 1e-4
        dpsi = (oracle.phase(th, f + h) - oracle.phase(th, f - h)) / (2 * h)
        tau_n = 5.0 * Ms / (256.0 * eta * v**8)
        series = (1 + (743.0 / 252 + 11.0 * eta / 3) * v**2 - 32.0 * math.pi / 5 * v**3
                  + (3058673.0 / 508032 + 5429.0 * eta / 504 + 617.0 * eta**2 / 72) * v**4)
        expect = 2 * math.pi * (tc - tau_n * series)
        rel = abs((dpsi - expect) / (2 * math.pi * tau_n))
        assert rel < 200 * v**5, (v, rel)


def test_exchange_symmetry_of_spin_terms():
    rng = np.random.default_rng(5)
    for _ in range(200):
        eta = rng.uniform(0.05, 0.25)
        x = math.sqrt(1 - 4 * eta)
        cs, ca = rng.uniform(-1, 1, 2)
        Ms, f = 2e-4, rng.uniform(20, 500)
        a = oracle.pn_coeffs(eta, x, cs, ca, Ms, f)
        b = oracle.pn_coeffs(eta, -x, cs, -ca, Ms, f)
        np.testing.assert_allclose(a, b, rtol=1e-13, atol=1e-10)


def test_spin_orbit_and_spin_spin_identities():
    rng = np.random.default_rng(7)
    for _ in range(300):
        q = rng.uniform(0.1, 1.0)
        c1, c2 = rng.uniform(-1, 1, 2)
        eta = _eta(q)
        m1 = 1.0 / (1 + q)
        m2 = q / (1 + q)
        x = m1 - m2
        cs, ca = 0.5 * (c1 + c2), 0.5 * (c1 - c2)
        Ms, f = 3e-4, 50.0
        phi = oracle.pn_coeffs(eta, x, cs, ca, Ms, f)
        phi0 = oracle.pn_coeffs(eta, x, 0.0, 0.0, Ms, f)
        beta = (c1 * (113 * m1**2 + 75 * eta) + c2 * (113 * m2**2 + 75 * eta)) / 12.0
        sigma = 79.0 / 8.0 * eta * c1 * c2 + 81.0 / 16.0 * (m1**2 * c1**2 + m2**2 * c2**2)
        assert abs(phi[3] - (-16 * math.pi + 4 * beta)) < 1e-11
        assert abs((phi[4] - phi0[4]) - (-10 * sigma)) < 1e-10
        assert phi[1] == 0.0 and phi[0] == 1.0


def test_phase_linear_in_tc_and_phic():
    th = _theta(tc=0.0, phic=0.0)
    f = 123.4
    base = oracle.phase(th, f)
    th2 = th.copy(); th2[10] = 0.05; th2[9] = 0.7
    assert abs(oracle.phase(th2, f) - (base + 2 * math.pi * f * 0.05 - 1.4)) < 1e-9


def test_amplitude_scaling():
    th = _theta()
    a = oracle.amplitude(th)
    th2 = th.copy(); th2[4] *= 2
    assert abs(oracle.amplitude(th2) * 2 / a - 1) < 1e-15
    th3 = th.copy(); th3[0] *= 2
    assert abs(oracle.amplitude(th3) / a / 2 ** (5 / 6) - 1) < 1e-14
