"""Pins for the oracle's Whittle log-likelihood ratio (Sec. 3.3 and 4.1.1 of
the paper: the standard frequency-domain likelihood with use_ratio).

* Zero noise: log Lambda(theta_inj) = rho^2 / 2 and no parameter vector
  exceeds it (Cauchy-Schwarz on the noise-weighted inner product).
* The optimal SNR of a Newtonian-amplitude signal matches the continuum
  formula rho^2 = (5/6) pi^(-4/3) (G Mc/c^3)^(5/3) (c/dL)^2 int f^(-7/3)/S df
  (Finn & Chernoff 1993; Cutler & Flanagan 1994) once the sum over bins is
  corrected to the trapezoid rule.
* Symmetries: psi -> psi + pi and phi_c -> phi_c + pi leave the strain
  unchanged.
* Noise: <n|n> averages 2 N per detector, and log Lambda(theta_inj) over
  noise realisations is N(rho^2/2, rho^2).
"""
import math

import numpy as np
import pytest
from scipy import integrate

import oracle
from paper_2509_04336_amd import inputs

TSUN = 1.32712440018e20 / 299792458.0**3
MPC = 3.0856775814913673e22
C_SI = 299792458.0


@pytest.fixture(scope="module")
def tiny():
    return oracle.build_event(inputs.tiny_event())


@pytest.fixture(scope="module")
def paper0():
    return oracle.build_event(inputs.paper_event(with_noise=False))


def test_max_likelihood_at_injection_zero_noise(tiny, paper0):
    for ev, th, _ in (tiny, paper0):
        assert abs(oracle.loglike_theta(ev, th) - 200.0) < 1e-9
        assert abs(oracle.optimal_snr2(ev, th) - 400.0) < 1e-9


def test_cauchy_schwarz_bound(tiny, paper0):
    rng = np.random.default_rng(11)
    for ev, th, _ in (tiny, paper0):
        u = rng.random((3000 if ev.n_det == 1 else 300, ev.ndim))
        L = oracle.loglike_batch_u(ev, u)
        assert np.all(L <= 200.0 + 1e-9)
        assert np.all(np.isfinite(L))


def test_continuum_snr_formula():
    spec = inputs.tiny_event()
    ev = oracle.event_from_spec(spec)
    th = spec.theta_inj.copy()
    th[4] = 800.0
    disc = oracle.optimal_snr2(ev, th)
    g = lambda f: f ** (-7.0 / 3.0) / inputs.psd_aligo(np.array([f]))[0]
    f0 = spec.f_lo
    f1 = spec.f_lo + (spec.n_bins - 1) * spec.df
    integral, _ = integrate.quad(g, f0, f1, epsabs=0, epsrel=1e-12, limit=500)
    trap = integral + 0.5 * spec.df * (g(f0) + g(f1))
    pref = 5.0 / 6.0 * math.pi ** (-4.0 / 3.0) * (th[0] * TSUN) ** (5.0 / 3.0) * (C_SI / (th[4] * MPC)) ** 2
    assert abs(disc / (pref * trap) - 1.0) < 2e-6


def test_polarisation_and_phase_symmetries(paper0):
    ev, th, _ = paper0
    rng = np.random.default_rng(2)
    for _ in range(20):
        u = rng.random(11)
        t = oracle.prior_transform(ev, u)
        L = oracle.loglike_theta(ev, t)
        t2 = t.copy(); t2[8] += math.pi
        t3 = t.copy(); t3[9] += math.pi
        assert abs(oracle.loglike_theta(ev, t2) - L) < 1e-8 * max(1, abs(L))
        assert abs(oracle.loglike_theta(ev, t3) - L) < 1e-8 * max(1, abs(L))


def test_invalid_parameters_give_minus_inf(paper0):
    ev, th, _ = paper0
    for j, v in ((1, 0.0), (1, 1.5), (4, -1.0), (0, float("nan"))):
        t = th.copy(); t[j] = v
        assert oracle.loglike_theta(ev, t) == -math.inf


def test_noise_statistics():
    spec = inputs.paper_event(with_noise=False)
    nn = []
    for seed in range(40):
        n = inputs.noise(seed, 0, 3, spec.psd, spec.df)
        nn.append(4 * spec.df * np.sum(np.abs(n) ** 2 / spec.psd, axis=1))
    nn = np.array(nn)
    N = spec.n_bins
    # <n|n> = sum of 2N unit-variance squares: mean 2N, std 2 sqrt(N)
    assert np.all(np.abs(nn.mean(axis=0) - 2 * N) < 4 * 2 * math.sqrt(N) / math.sqrt(40))


@pytest.mark.slow
def test_loglike_at_injection_over_noise():
    vals = []
    for seed in range(24):
        ev, th, _ = oracle.build_event(inputs.tiny_event().__class__(
            **{**inputs.tiny_event().__dict__,
               "noise": inputs.noise(seed, 0, 1, inputs.tiny_event().psd, 0.25)}))
        vals.append(oracle.loglike_theta(ev, th))
    vals = np.array(vals)
    # log Lambda(theta_inj) = rho^2/2 + <n|h> with <n|h> ~ N(0, rho^2), rho = 20
    assert abs(vals.mean() - 200.0) < 4 * 20.0 / math.sqrt(len(vals))
    assert 10.0 < vals.std(ddof=1) < 32.0
