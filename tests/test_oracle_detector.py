"""Pins for the oracle's detector response (antenna patterns, time delays).

* For a detector at the north pole with arms along x and y, F+^2 + Fx^2 has
  the polarisation-independent textbook form
  (1 + cos^2 t)^2 cos^2(2 p) / 4 + cos^2 t sin^2(2 p)  (t, p the polar and
  azimuthal angle of the source; Thorne 1987).
* F+^2 + Fx^2 does not depend on psi; psi -> psi + pi/2 flips both signs.
* A source at the zenith of an L-shaped detector has F+^2 + Fx^2 = 1.
* Time delays: a source overhead arrives R/c early, an antipodal one R/c late.
"""
import math

import numpy as np

import oracle
from paper_2509_04336_amd import inputs

POLE = (0.5 * (np.outer([1, 0, 0], [1, 0, 0]) - np.outer([0, 1, 0], [0, 1, 0]))).reshape(9)


def test_pole_detector_closed_form():
    rng = np.random.default_rng(3)
    for _ in range(500):
        ra, dec, psi = rng.uniform(0, 2 * math.pi), rng.uniform(-1.5, 1.5), rng.uniform(0, math.pi)
        fp, fx = oracle.antenna(POLE, ra, dec, psi)
        t = math.pi / 2 - dec
        p = ra
        exp = (1 + math.cos(t) ** 2) ** 2 * math.cos(2 * p) ** 2 / 4 + math.cos(t) ** 2 * math.sin(2 * p) ** 2
        assert abs(fp * fp + fx * fx - exp) < 1e-13


def test_polarisation_rotation():
    tens, _ = inputs.detector_geometry(3)
    rng = np.random.default_rng(4)
    for _ in range(300):
        D = tens[rng.integers(3)]
        ra, dec, psi = rng.uniform(0, 2 * math.pi), rng.uniform(-1.5, 1.5), rng.uniform(0, math.pi)
        fp, fx = oracle.antenna(D, ra, dec, psi, 0.3)
        fp2, fx2 = oracle.antenna(D, ra, dec, psi + 0.77, 0.3)
        fp3, fx3 = oracle.antenna(D, ra, dec, psi + math.pi / 2, 0.3)
        assert abs((fp**2 + fx**2) - (fp2**2 + fx2**2)) < 1e-13
        assert abs(fp + fp3) < 1e-13 and abs(fx + fx3) < 1e-13
        # rotation by psi mixes (F+, Fx) by the angle 2 psi
        c, s = math.cos(2 * 0.77), math.sin(2 * 0.77)
        assert abs(fp2 - (c * fp + s * fx)) < 1e-13 or abs(fp2 - (c * fp - s * fx)) < 1e-13


def test_zenith_and_delays():
    tens, locs = inputs.detector_geometry(3)
    R = inputs.EARTH_RADIUS_M
    c = 299792458.0
    for d in range(3):
        r = locs[d]
        dec = math.asin(r[2] / R)
        ra = math.atan2(r[1], r[0])
        for psi in (0.0, 0.4, 1.3):
            fp, fx = oracle.antenna(tens[d], ra, dec, psi)
            assert abs(fp * fp + fx * fx - 1.0) < 1e-12
        assert abs(oracle.time_delay(r, ra, dec) + R / c) < 1e-15
        assert abs(oracle.time_delay(r, ra + math.pi, -dec) - R / c) < 1e-15
    # delay differences are bounded by the baseline light travel time
    rng = np.random.default_rng(9)
    for _ in range(200):
        ra, dec = rng.uniform(0, 2 * math.pi), rng.uniform(-1.5, 1.5)
        dts = [oracle.time_delay(locs[d], ra, dec) for d in range(3)]
        for i in range(3):
            for j in range(3):
                assert abs(dts[i] - dts[j]) <= np.linalg.norm(locs[i] - locs[j]) / c + 1e-15


def test_gmst_is_a_rotation_in_ra():
    tens, locs = inputs.detector_geometry(3)
    a = oracle.antenna(tens[1], 1.0, 0.3, 0.2, gmst=0.5)
    b = oracle.antenna(tens[1], 0.5, 0.3, 0.2, gmst=0.0)
    assert abs(a[0] - b[0]) < 1e-14 and abs(a[1] - b[1]) < 1e-14
