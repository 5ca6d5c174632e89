"""Pins for the oracle's TaylorF2 phase and amplitude.

* Low-frequency limit: the phase tends to the Newtonian (0PN) closed form
  (3/128)(pi Mc f)^(-5/3), which depends on the chirp mass only; the first
  correction is O(v^2) (no 0.5PN term).
* Stationary-phase consistency: dPsi/df = 2 pi (t_c - tau(f)) with tau the
  TaylorT2 time to coalescence through 3.5PN for non-spinning binaries
  (Blanchet 2014, Living Rev. Relativ. 17:2), checked in integral form at
  velocities where every order matters.
* Test-mass limit: the spin-orbit terms (1.5, 2.5, 3, 3.5PN) and the 2PN
  spin-spin term at leading order in eta, from the Kerr circular-orbit
  energy and the test-mass flux.
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


GAMMA_E = 0.5772156649015329


def _taylor_t2(v, eta):
    """Time to coalescence over its Newtonian value, 5 M / (256 eta v^8),
    for a non-spinning binary through 3.5PN (the TaylorT2 series as given
    by Blanchet, Living Rev. Relativ. 17:2 (2014), with x = v^2)."""
    pi = math.pi
    t6 = (-10052469856691.0 / 23471078400 + 128 * pi**2 / 3 + 6848 * GAMMA_E / 105
          + (3147553127.0 / 3048192 - 451 * pi**2 / 12) * eta - 15211 * eta**2 / 1728
          + 25565 * eta**3 / 1296 + 3424.0 / 105 * np.log(16 * v * v))
    return (1 + (743 / 252 + 11 * eta / 3) * v**2 - 32 * pi / 5 * v**3
            + (3058673 / 508032 + 5429 * eta / 504 + 617 * eta**2 / 72) * v**4
            - (7729 / 252 - 13 * eta / 3) * pi * v**5 + t6 * v**6
            + (-15419335 / 127008 - 75703 * eta / 756 + 14809 * eta**2 / 378) * pi * v**7)


@pytest.mark.parametrize("q", [1.0, 0.6, 0.25])
def test_stationary_phase_time_relation(q):
    """Psi(f2) - Psi(f1) = 2 pi int t(f) df for the non-spinning phase at
    v = 0.12 ... 0.32, where every PN order up to 3.5PN moves the phase by far
    more than the tolerance (the 3.5PN term alone by about 1 rad at v = 0.3):
    a dropped, mis-signed or mis-indexed term of any phi_j fails."""
    mc, tc = 25.0, 0.013
    th = _theta(mc=mc, q=q, tc=tc)
    eta = _eta(q)
    Ms = _Ms(mc, q)
    xg, wg = np.polynomial.legendre.leggauss(40)
    for v1, v2 in ((0.12, 0.16), (0.2, 0.24), (0.28, 0.32)):
        f1, f2 = v1**3 / (math.pi * Ms), v2**3 / (math.pi * Ms)
        fm, fh = 0.5 * (f1 + f2), 0.5 * (f2 - f1)
        fs = fm + fh * xg
        vs = (math.pi * Ms * fs) ** (1.0 / 3.0)
        t = tc - 5 * Ms / (256 * eta * vs**8) * _taylor_t2(vs, eta)
        want = 2 * math.pi * fh * np.sum(wg * t)
        got = oracle.phase(th, f2) - oracle.phase(th, f1)
        assert abs(got - want) <= 1e-11 * abs(want) + 1e-12, (v1, got, want)


# Truncated power series in v (coefficient arrays of length _NS).
_NS = 10


def _smul(a, b):
    c = np.zeros(_NS)
    for i in range(_NS):
        c[i:] += a[i] * b[:_NS - i]
    return c


def _sinv(a):
    b = np.zeros(_NS)
    b[0] = 1.0 / a[0]
    for n in range(1, _NS):
        b[n] = -np.dot(a[1:n + 1], b[n - 1::-1][:n]) / a[0]
    return b


def _spow(a, alpha):
    """a^alpha for a[0] = 1 (J. C. P. Miller's recurrence)."""
    b = np.zeros(_NS)
    b[0] = 1.0
    for n in range(1, _NS):
        b[n] = sum((alpha * k - (n - k)) * a[k] * b[n - k] for k in range(1, n + 1)) / n
    return b


def test_spin_terms_test_mass_limit():
    """eta -> 0 with the heavy body spinning (chi1 = a, chi2 = 0): the phase
    coefficients follow from the energy of circular equatorial Kerr orbits
    (Bardeen, Press & Teukolsky 1972), E/mu = (1 - 2 w^2 + a w^3) /
    sqrt(1 - 3 w^2 + 2 a w^3) - 1 with w^2 = M/r and M Omega = w^3/(1 + a w^3),
    and the test-mass flux through 3.5PN (Tagoshi, Shibata, Tanaka & Sasaki
    1996): dt/dv = -(dE/dv)/F and dPsi/df = 2 pi t.  Pins the spin-orbit
    terms of phi3, phi5, phi6 and phi7 and the spin-spin term of phi4 at
    leading order in eta (their eta-dependent parts are not reached by this
    limit), and the eta -> 0 values of the non-spinning coefficients."""
    pi = math.pi
    for a in (-0.9, -0.3, 0.4, 0.95):
        w = np.zeros(_NS)
        w[1] = 1.0
        for _ in range(4):  # w(v) = v (1 + a w^3)^(1/3), v = (M Omega)^(1/3)
            w3 = _smul(_smul(w, w), w)
            t = a * w3
            t[0] += 1.0
            w = np.concatenate([[0.0], _spow(t, 1.0 / 3.0)[:_NS - 1]])
        num = np.zeros(_NS); num[0] = 1.0; num[2] = -2.0; num[3] = a
        den = np.zeros(_NS); den[0] = 1.0; den[2] = -3.0; den[3] = 2 * a
        e_w = _smul(num, _spow(den, -0.5))
        e_w[0] -= 1.0
        e = np.zeros(_NS)  # E(v) = e_w(w(v))
        wp = np.zeros(_NS); wp[0] = 1.0
        for k in range(_NS):
            e += e_w[k] * wp
            wp = _smul(wp, w)
        assert abs(e[2] + 0.5) < 1e-14 and abs(e[4] - 0.375) < 1e-14
        de = np.array([(k + 1) * e[k + 1] for k in range(_NS - 1)] + [0.0])
        mde = np.concatenate([-de[1:], [0.0]])  # -E'(v)/v
        for vv in (0.08, 0.2):
            lnv = math.log(vv)
            F = np.zeros(_NS)
            F[0] = 1.0
            F[2] = -1247 / 336
            F[3] = 4 * pi - 11 / 4 * a
            F[4] = -44711 / 9072 + 33 / 16 * a**2
            F[5] = -8191 / 672 * pi - 59 / 16 * a
            F6c = (6643739519 / 69854400 - 1712 / 105 * GAMMA_E + 16 / 3 * pi**2
                   - 3424 / 105 * math.log(2) - 65 / 6 * pi * a + 611 / 504 * a**2)
            F[7] = -16285 / 504 * pi + 162035 / 3888 * a + 65 / 8 * pi * a**2 - 71 / 24 * a**3
            # the log term of F6 is handled by linearity: coefficient series
            # with and without it
            F[6] = F6c
            c0 = _smul(mde, _sinv(F))
            F[6] = F6c - 1712 / 105
            c1 = _smul(mde, _sinv(F))
            a6c, a6l = c0[6], c1[6] - c0[6]  # a6 = a6c + a6l ln v
            tau = {j: 8 * c0[j] / (8 - j) for j in (2, 3, 4, 5, 7)}
            want = {j: 5 * tau[j] / (5 - j) for j in (2, 3, 4, 7)}
            want5c = -5.0 / 3.0 * tau[5]
            tau6c, tau6l = 8 * (a6c / 2 + a6l / 4), 4 * a6l
            Q = -5 * tau6l
            P = -5 * tau6c - Q
            Ms = 1e-4
            f = vv**3 / (pi * Ms)
            # oracle at eta = 0 (x = 1), chi_s = chi_a = a / 2; the SPA phase's
            # 3PN spin-spin, 3.5PN spin-spin and cubic terms are not part of it
            phi = oracle.pn_coeffs(0.0, 1.0, a / 2, a / 2, Ms, f)
            want[7] -= 14585 / 24 * a**3 - 815 / 2 * pi * a**2
            want6 = P + Q * lnv - 75515 / 288 * a**2
            for j in (2, 3, 4, 7):
                assert abs(phi[j] - want[j]) < 1e-9 * max(1.0, abs(want[j])), (a, j, phi[j], want[j])
            assert abs(phi[5] / (1 + 3 * lnv) - want5c) < 1e-9 * abs(want5c), (a, phi[5], want5c)
            assert abs(phi[6] - want6) < 1e-9 * abs(want6), (a, phi[6], want6)


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
