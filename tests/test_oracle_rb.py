"""Pins of the oracle's heterodyned (relative-binning) likelihood against the
exact Whittle likelihood of the same oracle.

Relative binning keeps the fiducial phase factor exact and interpolates the
ratio e^{-i (Phi - Phi0)} linearly between nodes, so it must reproduce the
exact likelihood wherever that ratio is linear in frequency inside every bin:

* at the fiducial point (ratio 1);
* with one sample per bin (the interpolation is only ever evaluated at a node);
* for parameters that differ from the fiducial only in coalescence phase and
  distance (ratio constant: a phase factor and an amplitude factor).

Elsewhere it is an approximation whose error falls as the bins are refined.
"""
import dataclasses

import numpy as np
import pytest

import oracle
from paper_2509_04336_amd import inputs


def _paper_rb(n_rb_bins, edges=None):
    spec = inputs.paper_event(seed=0)
    ev0, th, data = oracle.build_event(spec)
    spec = dataclasses.replace(spec, fixed_theta=np.array(ev0._keep["fixed_theta"]))
    rspec = inputs.rb_event(spec, th, n_rb_bins)
    if edges is not None:
        rspec = dataclasses.replace(rspec, rb_edges=np.asarray(edges, dtype=np.int32))
    ev = oracle.event_from_spec(rspec, data)
    return ev, th, spec


def test_rb_equals_exact_at_the_fiducial_point():
    ev, th, _ = _paper_rb(63)
    exact = oracle.loglike_theta(ev, th)
    rb = oracle.loglike_rb(ev, th)
    assert abs(rb - exact) <= 1e-9 * max(1.0, abs(exact))


def test_rb_with_one_sample_per_bin_is_exact_anywhere():
    spec = inputs.tiny_event()
    ev0, th, data = oracle.build_event(spec)
    spec = dataclasses.replace(spec, fixed_theta=np.array(ev0._keep["fixed_theta"]))
    rspec = dataclasses.replace(spec, like_kind=2, rb_theta0=th,
                                rb_edges=np.arange(spec.n_bins + 1, dtype=np.int32))
    ev = oracle.event_from_spec(rspec, data)
    rng = np.random.default_rng(3)
    for _ in range(4):
        u = rng.uniform(size=spec.ndim)
        thp = oracle.prior_transform(ev, u)
        exact = oracle.loglike_theta(ev, thp)
        rb = oracle.loglike_rb(ev, thp)
        assert abs(rb - exact) <= 1e-9 * max(1.0, abs(exact)), (exact, rb)


def test_rb_is_exact_for_phase_and_distance_changes():
    ev, th, _ = _paper_rb(31)
    for dphi, dscale in ((0.7, 1.0), (0.0, 1.37), (-2.1, 0.6)):
        thp = th.copy()
        thp[9] += dphi
        thp[4] *= dscale
        exact = oracle.loglike_theta(ev, thp)
        rb = oracle.loglike_rb(ev, thp)
        assert abs(rb - exact) <= 1e-9 * max(1.0, abs(exact)), (dphi, dscale, exact, rb)


def test_rb_error_is_small_near_the_fiducial_and_falls_with_finer_bins():
    """Posterior-scale perturbations (log L within ~1 of its fiducial value):
    the interpolation error is second order in the bin width, so quadrupling
    the bins must cut it by well over 4 (16 in the limit)."""
    coarse, th, _ = _paper_rb(63)
    fine, _, _ = _paper_rb(255)
    rng = np.random.default_rng(5)
    worst = {63: 0.0, 255: 0.0}
    for _ in range(6):
        thp = th.copy()
        thp[0] *= 1.0 + 2e-4 * rng.standard_normal()    # chirp mass
        thp[1] = min(1.0, thp[1] * (1.0 + 5e-3 * rng.standard_normal()))
        thp[2] += 5e-3 * rng.standard_normal()
        thp[10] += 2e-4 * rng.standard_normal()          # t_c [s]
        thp[6] += 2e-3 * rng.standard_normal()           # ra
        exact = oracle.loglike_theta(coarse, thp)
        for ev, nb in ((coarse, 63), (fine, 255)):
            worst[nb] = max(worst[nb], abs(oracle.loglike_rb(ev, thp) - exact))
    assert worst[255] < 0.02, worst
    assert worst[255] < worst[63] / 4.0, worst


def test_rb_event_validation():
    spec = inputs.tiny_event()
    with pytest.raises(ValueError):
        oracle.event_from_spec(dataclasses.replace(spec, like_kind=2, rb_theta0=None,
                                                   rb_edges=np.array([0, spec.n_bins])))
    with pytest.raises(ValueError):
        oracle.event_from_spec(dataclasses.replace(
            spec, like_kind=2, rb_theta0=np.zeros(11), rb_edges=np.array([0, 5, 5, spec.n_bins])))


@pytest.mark.parametrize("n,nb", [(945, 31), (4017, 255), (4017, 63), (100, 200)])
def test_rb_nodes_are_valid_sample_indices(n, nb):
    e = inputs.rb_edges(20.0, 0.25, n, nb)
    assert e[0] == 0 and e[-1] == n
    assert np.all(np.diff(e) > 0)
    assert len(e) - 1 <= min(nb, n)
    # narrower bins at low frequency, where the phase varies fastest
    if n > 1000:
        w = np.diff(e)
        assert w[0] < w[len(w) // 2]
