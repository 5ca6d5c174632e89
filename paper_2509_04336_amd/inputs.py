"""Seeded synthetic inputs for the acceptance-walk nested sampler.

This module builds the *inputs* of the method and nothing of its arithmetic:
frequency grids, an analytic noise power spectral density, coloured Gaussian
noise draws, detector geometry, injection parameter tables, prior ranges and
the sampler settings of each workload.  It never evaluates a waveform or a
likelihood; callers add the injected signal themselves (the HIP library's
``signal`` entry point on the product path, the CPU oracle in tests).

Both the oracle and the HIP path are fed from here, and from nowhere else.

Workloads (synthetic stand-ins for the paper's bilby/O4 injections, which are
not available; shapes follow Sec. 4.1-4.3 of the paper):

* ``tiny``      4-D (Mc, q, chi1, chi2), one detector with fixed antenna
                (F+ = 1, Fx = 0, no delay), 4 s at 20-256 Hz (945 bins), zero
                noise, SNR 20, 100 live points, 50 deleted per batch.
* ``paper``     11-D aligned-spin BBH, three L-shaped detectors, 4 s at
                20-1024 Hz (4017 bins), Gaussian noise, SNR 20, 1000 live
                points, 500 deleted per batch (Sec. 4.1.1 settings).
* ``long``      the tiny workload at 8 s, 20-2048 Hz (16225 bins).
* ``multi``     64 independent 11-D events of 4-64 s (4017-64257 bins).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

PARAM_NAMES = ("chirp_mass", "mass_ratio", "chi_1", "chi_2", "luminosity_distance",
               "theta_jn", "ra", "dec", "psi", "phase", "geocent_time")
NPAR = 11
PERIODIC_11D = (6, 8, 9)  # ra, psi, phase wrap in the unit cube (Sec. 4.1.1)

EARTH_RADIUS_M = 6.371e6

# Injection of the 4-s signal (Table 2 of the paper), parameter order above.
TABLE2_INJECTION = np.array([35.0, 0.90, 0.40, -0.30, 1000.0, 0.40, 1.38, -1.21, 2.66, 1.30, 0.0])
# Injection of the 8-s signal (Table 4 of the paper).
TABLE4_INJECTION = np.array([10.0, 0.70, -0.34, 0.01, 500.0, 1.30, 1.07, -1.01, 1.83, 5.21, 0.0])

# Prior ranges (Table 1 for the extrinsic parameters; Sec. 4.1.1 for the
# 4-s intrinsic ranges; the tiny workload uses Mc 20-40, q 0.25-1, chi +-0.9).
_EXTRINSIC_LO = [100.0, 0.0, 0.0, -math.pi / 2, 0.0, 0.0, -0.1]
_EXTRINSIC_HI = [5000.0, math.pi, 2 * math.pi, math.pi / 2, math.pi, 2 * math.pi, 0.1]
PRIOR_TINY_LO = np.array([20.0, 0.25, -0.9, -0.9] + _EXTRINSIC_LO)
PRIOR_TINY_HI = np.array([40.0, 1.0, 0.9, 0.9] + _EXTRINSIC_HI)
PRIOR_PAPER_LO = np.array([25.0, 0.25, -1.0, -1.0] + _EXTRINSIC_LO)
PRIOR_PAPER_HI = np.array([50.0, 1.0, 1.0, 1.0] + _EXTRINSIC_HI)


def grid(duration: float, f_lo: float, f_hi: float):
    """Uniform frequency grid f_k = f_lo + k/T, k = 0..N-1, N = T (f_hi - f_lo) + 1."""
    df = 1.0 / duration
    n = int(round((f_hi - f_lo) * duration)) + 1
    return f_lo, df, n


def frequencies(f_lo: float, df: float, n: int) -> np.ndarray:
    return f_lo + np.arange(n, dtype=np.float64) * df


def psd_aligo(f: np.ndarray, s0: float = 1e-49, f0: float = 215.0) -> np.ndarray:
    """Analytic Advanced-LIGO noise fit (Sathyaprakash & Schutz 2009, Living
    Rev. Relativ. 12:2), one-sided, 1/Hz.  Stands in for the O4 design curves."""
    x = np.asarray(f, dtype=np.float64) / f0
    return s0 * (x ** -4.14 - 5.0 * x ** -2 + 111.0 * (1.0 - x ** 2 + 0.5 * x ** 4) / (1.0 + 0.5 * x ** 2))


def noise(seed: int, event: int, n_det: int, psd: np.ndarray, df: float) -> np.ndarray:
    """Coloured Gaussian noise n_{d,k} = sqrt(S_d(f_k) / (4 df)) (a + i b),
    a, b ~ N(0, 1) from numpy's default generator seeded [seed, event, d].
    Returns complex128 [n_det, n_bins]; E<n|n> = 2 N per detector."""
    psd = np.atleast_2d(psd)
    out = np.empty(psd.shape, dtype=np.complex128)
    for d in range(n_det):
        rng = np.random.default_rng([seed, event, d])
        a = rng.standard_normal(psd.shape[1])
        b = rng.standard_normal(psd.shape[1])
        out[d] = np.sqrt(psd[d] / (4.0 * df)) * (a + 1j * b)
    return out


# Synthetic three-detector network: 90-degree L-shaped interferometers at
# (latitude, longitude, x-arm azimuth from north towards east) in degrees,
# on a spherical Earth; the y arm is the x arm rotated by -90 degrees.
# H/L/V-inspired placements, not the surveyed observatory geometry.
DETECTOR_SITES = (
    ("A", 46.455, -119.408, 36.0),
    ("B", 30.563, -90.774, 108.0),
    ("C", 43.631, 10.504, 19.0),
)


def _local_frame(lat_deg: float, lon_deg: float):
    la, lo = math.radians(lat_deg), math.radians(lon_deg)
    east = np.array([-math.sin(lo), math.cos(lo), 0.0])
    north = np.array([-math.sin(la) * math.cos(lo), -math.sin(la) * math.sin(lo), math.cos(la)])
    up = np.array([math.cos(la) * math.cos(lo), math.cos(la) * math.sin(lo), math.sin(la)])
    return east, north, up


def detector_geometry(n_det: int = 3):
    """Response tensors D = (x x^T - y y^T)/2 [n_det, 9] and Earth-fixed
    positions [n_det, 3] (m) of the synthetic network."""
    tensors, locs = [], []
    for name, lat, lon, az in DETECTOR_SITES[:n_det]:
        east, north, up = _local_frame(lat, lon)
        ax = math.radians(az)
        ay = math.radians(az - 90.0)
        x = math.cos(ax) * north + math.sin(ax) * east
        y = math.cos(ay) * north + math.sin(ay) * east
        tensors.append((0.5 * (np.outer(x, x) - np.outer(y, y))).reshape(9))
        locs.append(EARTH_RADIUS_M * up)
    return np.array(tensors), np.array(locs)


@dataclasses.dataclass
class EventSpec:
    """Everything an event needs except the injected signal."""
    f_lo: float
    df: float
    n_bins: int
    n_det: int
    ndim: int
    psd: np.ndarray                      # [n_det, n_bins]
    noise: np.ndarray                    # complex [n_det, n_bins] (zeros for zero noise)
    det_tensor: Optional[np.ndarray]     # [n_det, 9] or None
    det_loc: Optional[np.ndarray]        # [n_det, 3] or None
    fixed_antenna: Optional[np.ndarray]  # [n_det, 2] or None
    prior_lo: np.ndarray                 # [11]
    prior_hi: np.ndarray                 # [11]
    fixed_theta: np.ndarray              # [11]; entry 4 (dL) is rescaled for the SNR
    theta_inj: np.ndarray                # [11] before SNR rescaling of dL
    target_snr: float
    gmst: float = 0.0
    like_kind: int = 0                   # 0 GW likelihood, 1 Gaussian toy, 2 GW relative binning
    toy_sigma: float = 0.1
    rb_theta0: Optional[np.ndarray] = None   # [11] fiducial parameters (like_kind 2)
    rb_edges: Optional[np.ndarray] = None    # [B + 1] node sample indices (like_kind 2)


@dataclasses.dataclass
class SamplerSpec:
    n_live: int
    num_delete: int
    naccept: int
    maxmcmc: int
    walk0: int = 100
    term_kind: int = 0     # 0: dlogZ < thr (bilby default), 1: log(Z_live/Z) < log(thr)
    term_thr: float = 0.1

    @property
    def delay(self) -> float:
        return max(self.n_live / 10.0 - 1.0, 0.0)


def tiny_event(duration: float = 4.0, f_hi: float = 256.0, snr: float = 20.0) -> EventSpec:
    f_lo, df, n = grid(duration, 20.0, f_hi)
    f = frequencies(f_lo, df, n)
    psd = psd_aligo(f)[None, :]
    theta = TABLE2_INJECTION.copy()
    theta[5] = 0.0   # face-on
    theta[9] = 0.0
    theta[10] = 0.0
    return EventSpec(f_lo=f_lo, df=df, n_bins=n, n_det=1, ndim=4, psd=psd,
                     noise=np.zeros((1, n), np.complex128), det_tensor=None, det_loc=None,
                     fixed_antenna=np.array([[1.0, 0.0]]), prior_lo=PRIOR_TINY_LO.copy(),
                     prior_hi=PRIOR_TINY_HI.copy(), fixed_theta=theta.copy(), theta_inj=theta,
                     target_snr=snr)


def paper_event(duration: float = 4.0, f_hi: float = 1024.0, snr: float = 20.0, seed: int = 0,
                event: int = 0, theta: Optional[np.ndarray] = None, with_noise: bool = True
                ) -> EventSpec:
    f_lo, df, n = grid(duration, 20.0, f_hi)
    f = frequencies(f_lo, df, n)
    psd = np.repeat(psd_aligo(f)[None, :], 3, axis=0)
    tens, locs = detector_geometry(3)
    th = TABLE2_INJECTION.copy() if theta is None else np.asarray(theta, np.float64).copy()
    nz = noise(seed, event, 3, psd, df) if with_noise else np.zeros((3, n), np.complex128)
    return EventSpec(f_lo=f_lo, df=df, n_bins=n, n_det=3, ndim=11, psd=psd, noise=nz,
                     det_tensor=tens, det_loc=locs, fixed_antenna=None,
                     prior_lo=PRIOR_PAPER_LO.copy(), prior_hi=PRIOR_PAPER_HI.copy(),
                     fixed_theta=th.copy(), theta_inj=th, target_snr=snr)


def toy_event(ndim: int, sigma: float) -> EventSpec:
    """Gaussian toy in the unit cube; the event carries no strain data."""
    lo = np.zeros(NPAR)
    hi = np.ones(NPAR)
    return EventSpec(f_lo=20.0, df=1.0, n_bins=1, n_det=1, ndim=ndim,
                     psd=np.ones((1, 1)), noise=np.zeros((1, 1), np.complex128),
                     det_tensor=None, det_loc=None, fixed_antenna=np.array([[1.0, 0.0]]),
                     prior_lo=lo, prior_hi=hi, fixed_theta=np.full(NPAR, 0.5),
                     theta_inj=np.full(NPAR, 0.5), target_snr=0.0, like_kind=1,
                     toy_sigma=sigma)


def multi_event_durations(n_events: int = 64, seed: int = 0):
    """Segment lengths for the multi-event workload, drawn per event from
    {4, 8, 16, 32, 64} s with numpy's generator seeded [seed, 4242]."""
    rng = np.random.default_rng([seed, 4242])
    return rng.choice(np.array([4.0, 8.0, 16.0, 32.0, 64.0]), size=n_events)


def multi_event_theta(event: int, seed: int = 0):
    """Injection for event e of the multi-event workload: u ~ U[0,1]^11 from
    numpy's generator seeded [seed, event, 777] (mapped to the prior by the
    caller), and the target SNR ~ U[10, 40]."""
    rng = np.random.default_rng([seed, event, 777])
    u = rng.random(NPAR)
    snr = 10.0 + 30.0 * rng.random()
    return u, snr


def multi_event_injection(event: int, seed: int = 0):
    """Physical injection for event e of the multi-event workload: every
    parameter uniform in the paper prior's box (an injection distribution, not
    the prior), from numpy's generator seeded [seed, event, 778], and the
    target SNR ~ U[10, 40]."""
    rng = np.random.default_rng([seed, event, 778])
    th = PRIOR_PAPER_LO + rng.random(NPAR) * (PRIOR_PAPER_HI - PRIOR_PAPER_LO)
    snr = 10.0 + 30.0 * rng.random()
    return th, snr


TINY_SAMPLER = SamplerSpec(n_live=100, num_delete=50, naccept=30, maxmcmc=5000)
PAPER_SAMPLER = SamplerSpec(n_live=1000, num_delete=500, naccept=60, maxmcmc=5000,
                            term_kind=1, term_thr=1e-3)
MULTI_SAMPLER = SamplerSpec(n_live=500, num_delete=250, naccept=60, maxmcmc=5000,
                            term_kind=1, term_thr=1e-3)


# ---------------------------------------------------------------------------
# Relative-binning nodes: a configuration of the heterodyned likelihood, like
# the frequency grid.  Nodes sit at equal steps of
#   Phi(f) = sum_g |f^g - f_lo^g| / |f_end^g - f_lo^g|,  g in {-5/3, -2/3, 1, 5/3, 7/3}
# (the power laws through which phase differences between waveforms grow
# along the band), rounded to sample indices; f_end = f_lo + n_bins df is the
# node one grid step past the last sample.
# ---------------------------------------------------------------------------
RB_POWERS = (-5.0 / 3.0, -2.0 / 3.0, 1.0, 5.0 / 3.0, 7.0 / 3.0)


def rb_edges(f_lo: float, df: float, n_bins: int, n_nodes_bins: int) -> np.ndarray:
    """Sample indices of n_nodes_bins + 1 nodes (fewer if rounding merges
    some), from 0 to n_bins, strictly increasing."""
    k = np.arange(n_bins + 1, dtype=np.float64)
    f = f_lo + k * df
    phi = np.zeros_like(f)
    for g in RB_POWERS:
        phi += np.abs(f ** g - f_lo ** g) / abs(f[-1] ** g - f_lo ** g)
    targets = np.linspace(0.0, phi[-1], n_nodes_bins + 1)
    idx = np.searchsorted(phi, targets)
    idx = np.clip(idx, 0, n_bins)
    idx[0], idx[-1] = 0, n_bins
    return np.unique(idx).astype(np.int32)


def rb_event(spec: EventSpec, theta0, n_nodes_bins: int) -> EventSpec:
    """The same event with the heterodyned likelihood around theta0."""
    return dataclasses.replace(spec, like_kind=2, rb_theta0=np.array(theta0, dtype=np.float64),
                               rb_edges=rb_edges(spec.f_lo, spec.df, spec.n_bins, n_nodes_bins))

