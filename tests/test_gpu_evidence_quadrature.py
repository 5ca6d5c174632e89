"""Evidence of the GPU sampler on a real GW likelihood with a closed answer:
the 4-D workload with both spins pinned to the injection (prior bounds equal)
leaves a 2-D posterior in chirp mass and mass ratio whose log Z brute-force
quadrature on a fine grid gives to far better than the sampler's error
(Sec. 2.2: Z is the prior integral of L).  Both inner kernels, the
acceptance walk and hit-and-run slice sampling, must land on it."""
import dataclasses
import math

import numpy as np
import pytest

import oracle
from paper_2509_04336_amd import inputs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def slice_problem():
    spec = inputs.tiny_event(snr=12.0)
    ev0, th, data = oracle.build_event(spec)
    lo = spec.prior_lo.copy()
    hi = spec.prior_hi.copy()
    lo[2] = hi[2] = th[2]
    lo[3] = hi[3] = th[3]
    spec2 = dataclasses.replace(spec, prior_lo=lo, prior_hi=hi,
                                fixed_theta=np.array(ev0._keep["fixed_theta"]))
    ev = oracle.event_from_spec(spec2, data)

    def grid_L(u0, u1):
        U = np.zeros((len(u0) * len(u1), 4))
        U[:, 0] = np.repeat(u0, len(u1))
        U[:, 1] = np.tile(u1, len(u0))
        U[:, 2:] = 0.5
        return oracle.loglike_batch_u(ev, U).reshape(len(u0), len(u1))

    # coarse pass to bracket the chirp-mass support, then a fine midpoint grid
    c0 = (np.arange(300) + 0.5) / 300
    c1 = (np.arange(120) + 0.5) / 120
    Lc = grid_L(c0, c1)
    keep = np.where(Lc.max(axis=1) > Lc.max() - 60)[0]
    a0 = max(c0[keep.min()] - 2 / 300, 0.0)
    b0 = min(c0[keep.max()] + 2 / 300, 1.0)
    n0, n1 = 700, 400
    f0 = a0 + (np.arange(n0) + 0.5) * (b0 - a0) / n0
    f1 = (np.arange(n1) + 0.5) / n1
    Lf = grid_L(f0, f1)
    mx = Lf.max()
    logZ = mx + math.log(np.sum(np.exp(Lf - mx)) * (b0 - a0) / n0 / n1)
    return spec2, data, logZ


@pytest.mark.parametrize("inner,naccept", [("walk", 30), ("hrss", 20)])
def test_two_dimensional_gw_slice_evidence_against_quadrature(slice_problem, inner, naccept):
    from paper_2509_04336_amd import nsmi
    spec, data, logZ_quad = slice_problem
    vals = []
    for seed in range(8):
        with nsmi.Context([spec], [data], n_live=400, num_delete=200, naccept=naccept,
                          maxmcmc=5000, walk0=naccept, term_kind=1, term_thr=1e-3,
                          seed=600 + seed, inner=inner) as ctx:
            for _ in range(400):
                if ctx.converged():
                    break
                ctx.step()
            e = ctx.evidence()
            assert e["converged"]
            vals.append(e["logZ"])
    vals = np.array(vals)
    se = max(vals.std(ddof=1), 0.1) / math.sqrt(len(vals))
    print(f"{inner}: log Z {vals.mean():.4f} +- {se:.4f}, quadrature {logZ_quad:.4f}", flush=True)
    assert abs(vals.mean() - logZ_quad) < 4 * se + 0.05, (vals, logZ_quad)
