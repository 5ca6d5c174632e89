"""GPU parity: the HIP library against the CPU oracle on the same seeded
inputs, element by element.

Tolerances (FP64 path): per-call log-likelihood |dlogL| <= 1e-6 absolute;
unit-cube coordinates after walks within 1e-12 (the walk arithmetic is the
same sequence of IEEE operations on both sides, except the logarithm in the
differential-evolution scale, where device and host libm may differ by an
ulp); integer results (Philox words, accept/call/out-of-bounds counts, dead
counts, tuned walk lengths) exactly.
"""
import math
import sys

import numpy as np
import pytest

import oracle
from helpers import WORKLOADS, both_sides
from paper_2509_04336_amd import inputs

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _nsmi():
    from paper_2509_04336_amd import nsmi
    return nsmi


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _theta_draws(ev, n, seed):
    rng = np.random.default_rng(seed)
    u = rng.random((n, ev.ndim))
    return u, np.array([oracle.prior_transform(ev, x) for x in u])


@pytest.mark.parametrize("name", ["tiny", "paper", "long"])
def test_loglike_batch_matches_oracle(name):
    nsmi = _nsmi()
    ev, spec, data, th_inj = both_sides(WORKLOADS[name]())
    _say("loglike parity", name, spec.n_bins, spec.n_det)
    n = {"tiny": 777, "paper": 300, "long": 150}[name]
    u, th = _theta_draws(ev, n, 1)
    # points near the injection as well as prior draws
    near = th_inj[None, :] + 1e-3 * np.random.default_rng(2).standard_normal((20, 11)) * np.abs(th_inj + 1)
    near[:, 1] = np.clip(near[:, 1], 0.3, 1.0)
    th = np.vstack([th, th_inj[None, :], near])
    want = oracle.loglike_batch_theta(ev, th)
    with nsmi.Context([spec], [data], n_live=8, num_delete=4, naccept=5, maxmcmc=10, walk0=5) as ctx:
        t = torch.tensor(th, device="cuda")
        out = torch.empty(len(th), dtype=torch.float64, device="cuda")
        ctx.loglike_batch(0, t, out)
        got = out.cpu().numpy()
        uu = torch.tensor(u, device="cuda")
        out2 = torch.empty(len(u), dtype=torch.float64, device="cuda")
        ctx.loglike_batch_u(0, uu, out2)
        got_u = out2.cpu().numpy()
    err = np.abs(got - want)
    _say("max |dlogL|", err.max(), "at |logL|", np.abs(want).max())
    assert np.all(err <= 1e-6), (err.max(), np.argmax(err))
    assert np.all(np.abs(got_u - want[: len(u)]) <= 1e-6)
    if spec.target_snr > 0 and not spec.noise.any():
        assert abs(got[n] - 0.5 * spec.target_snr**2) < 1e-6


def test_loglike_invalid_parameters_and_empty_batch():
    nsmi = _nsmi()
    ev, spec, data, th = both_sides(WORKLOADS["tiny"]())
    bad = np.repeat(th[None, :], 4, axis=0)
    bad[0, 1] = 0.0
    bad[1, 1] = 1.2
    bad[2, 4] = -5.0
    bad[3, 0] = np.nan
    with nsmi.Context([spec], [data], n_live=8, num_delete=4, naccept=5, maxmcmc=10, walk0=5) as ctx:
        t = torch.tensor(bad, device="cuda")
        out = torch.zeros(4, dtype=torch.float64, device="cuda")
        ctx.loglike_batch(0, t, out)
        assert np.all(np.isneginf(out.cpu().numpy()))
        empty = torch.empty((0, 11), dtype=torch.float64, device="cuda")
        ctx.loglike_batch(0, empty, out)


@pytest.mark.parametrize("name", ["tiny", "paper"])
def test_signal_matches_oracle_waveform(name):
    nsmi = _nsmi()
    ev, spec, data, th = both_sides(WORKLOADS[name]())
    h_gpu = nsmi.signal(spec, th)
    h_or = oracle.waveform(ev, th)
    scale = np.abs(h_or).max()
    assert np.abs(h_gpu - h_or).max() <= 1e-10 * scale


@pytest.mark.parametrize("name", ["tiny", "paper", "toy4"])
def test_initial_live_set(name):
    nsmi = _nsmi()
    ev, spec, data, _ = both_sides(WORKLOADS[name]())
    n = 64 if name == "paper" else 100
    ns = oracle.NS(ev, n_live=n, naccept=10, maxmcmc=100, seed=42)
    with nsmi.Context([spec], [data], n_live=n, num_delete=n // 2, naccept=10, maxmcmc=100,
                      walk0=10, seed=42) as ctx:
        ug, Lg = ctx.live()
    uo, Lo = ns.live()
    assert np.array_equal(ug, uo)  # Philox words and 53-bit uniforms, bit for bit
    assert np.abs(Lg - Lo).max() <= 1e-6


def _run_pair(name, n_live, k, W, iters, seed, walk_fixed=True):
    nsmi = _nsmi()
    ev, spec, data, _ = both_sides(WORKLOADS[name]())
    naccept, maxmcmc = 20, 5000
    ns = oracle.NS(ev, n_live=n_live, naccept=naccept, maxmcmc=maxmcmc, walk0=W, seed=seed)
    ctx = nsmi.Context([spec], [data], n_live=n_live, num_delete=k, naccept=naccept,
                       maxmcmc=maxmcmc, walk0=W, seed=seed)
    uo, Lo = ns.live()
    ctx.set_live(0, uo, Lo)  # identical keys for the first selection
    for it in range(iters):
        _say(f"step parity {name} n={n_live} k={k} W={W} iter={it}")
        ns.step(k, W if walk_fixed else 0)
        ctx.step(k, W if walk_fixed else 0)
        ug, Lg = ctx.live()
        uo, Lo = ns.live()
        assert np.abs(ug - uo).max() <= 1e-12, np.abs(ug - uo).max()
        assert np.abs(Lg - Lo).max() <= 1e-6
        eg, eo = ctx.evidence(), ns.evidence()
        so = ns.stats()
        assert eg["last_accept"] == so["last_acc"]
        assert eg["last_calls"] == so["last_calls"]
        assert eg["n_oob"] == so["oob"]
        assert eg["W"] == ns.W
        assert eg["walk_capped"] == so["capped"]
        assert eg["batch"] == ns.batch
        assert abs(eg["logX"] - eo["logX"]) <= 1e-12
        assert abs(eg["logZ_dead"] - eo["logZ_dead"]) <= 1e-6
        assert abs(eg["H"] - eo["H"]) <= 1e-6
        assert abs(eg["logZ"] - eo["logZ"]) <= 1e-6
        assert abs(eg["logZ_err"] - eo["logZ_err"]) <= 1e-7
        assert np.array_equal(ctx.chain_stats()[:, :3], ns.last_chains())
    ud, Ld, lwd, nld = ctx.dead()
    uod, Lod, lwo, nlo = ns.dead()
    assert np.abs(ud - uod).max() <= 1e-12
    assert np.abs(Ld - Lod).max() <= 1e-6
    assert np.abs(lwd - lwo).max() <= 1e-12
    assert np.array_equal(nld, nlo)
    ctx.close()


def test_single_walk_step_parity():
    _run_pair("tiny", 100, 50, 1, 3, seed=7)


def test_walk_parity_tiny_many_steps():
    _run_pair("tiny", 100, 50, 60, 3, seed=8)


def test_walk_parity_tuned_lengths():
    _run_pair("tiny", 100, 50, 30, 4, seed=9, walk_fixed=False)


def test_walk_parity_paper_scale():
    _run_pair("paper", 200, 100, 12, 2, seed=10)


def test_walk_parity_paper_scale_long_walk():
    # 300 steps per chain: scans span several 64-step windows, windows are
    # drawn ahead by idle waves and evicted from the four window slots
    _run_pair("paper", 100, 50, 300, 1, seed=13)


def test_walk_parity_toy_extreme_batch():
    # k = n - 2 (largest legal batch) and k = 1 (sequential limit)
    _run_pair("toy4", 50, 48, 7, 3, seed=11)
    _run_pair("toy4", 50, 1, 7, 5, seed=12)


def test_step_argument_checks():
    nsmi = _nsmi()
    ev, spec, data, _ = both_sides(WORKLOADS["toy4"]())
    with nsmi.Context([spec], [data], n_live=20, num_delete=10, naccept=5, maxmcmc=50,
                      walk0=5) as ctx:
        for k, w in ((19, 1), (20, 1), (5, 51)):
            with pytest.raises(nsmi.NSError) as ei:
                ctx.step(k, w)
            assert ei.value.status == nsmi.NS_EINVAL


@pytest.mark.slow
def test_gaussian_toy_evidence_on_gpu():
    nsmi = _nsmi()
    from scipy.special import ndtr
    d, sigma = 4, 0.02
    spec = inputs.toy_event(d, sigma)
    exact = d * math.log(math.sqrt(2 * math.pi) * sigma * (ndtr(0.5 / sigma) - ndtr(-0.5 / sigma)))
    vals = []
    for seed in range(6):
        with nsmi.Context([spec], [np.zeros((1, 1))], n_live=400, num_delete=200, naccept=30,
                          maxmcmc=5000, walk0=50, term_kind=1, term_thr=1e-3, seed=seed) as ctx:
            for _ in range(400):
                if ctx.converged():
                    break
                ctx.step()
            vals.append(ctx.evidence()["logZ"])
    vals = np.array(vals)
    sem = vals.std(ddof=1) / math.sqrt(len(vals))
    _say("toy logZ", vals, "exact", exact)
    assert abs(vals.mean() - exact) < 3.5 * sem + 0.02


@pytest.mark.parametrize("name", ["tiny", "paper", "long"])
def test_mixed_precision_loglike_within_tolerance(name):
    """Mixed precision (FP64 phase and reduction, FP32 sin/cos and blocked
    FP32 accumulation) against the FP64 oracle: |dlogL| <= 1e-3 per call."""
    nsmi = _nsmi()
    ev, spec, data, th_inj = both_sides(WORKLOADS[name]())
    n = {"tiny": 777, "paper": 300, "long": 150}[name]
    u, th = _theta_draws(ev, n, 5)
    th = np.vstack([th, th_inj[None, :]])
    want = oracle.loglike_batch_theta(ev, th)
    with nsmi.Context([spec], [data], n_live=8, num_delete=4, naccept=5, maxmcmc=10, walk0=5) as ctx:
        t = torch.tensor(th, device="cuda")
        out = torch.empty(len(th), dtype=torch.float64, device="cuda")
        ctx.loglike_batch(0, t, out, precision=nsmi.NS_MIXED)
        got = out.cpu().numpy()
    err = np.abs(got - want)
    rel = err / np.maximum(np.abs(want), 1.0)
    _say(f"mixed {name}: max |dlogL| {err.max():.3e}, median {np.median(err):.3e}, "
         f"max rel {rel.max():.3e}, at injection {err[-1]:.3e}")
    assert err.max() <= 1e-3


def test_mixed_precision_walk_matches_fp64_statistically():
    """A mixed-precision run and an FP64 run of the tiny workload agree on
    log Z within their combined error."""
    nsmi = _nsmi()
    ev, spec, data, _ = both_sides(WORKLOADS["tiny"]())
    vals = {}
    for prec in (nsmi.NS_FP64, nsmi.NS_MIXED):
        zs = []
        for seed in range(3):
            with nsmi.Context([spec], [data], n_live=100, num_delete=50, naccept=30,
                              maxmcmc=5000, walk0=100, precision=prec, seed=seed) as ctx:
                for _ in range(300):
                    if ctx.converged():
                        break
                    ctx.step()
                e = ctx.evidence()
                assert e["converged"]
                zs.append((e["logZ"], e["logZ_err"]))
        vals[prec] = zs
    z64 = np.array([z for z, _ in vals[nsmi.NS_FP64]])
    zmx = np.array([z for z, _ in vals[nsmi.NS_MIXED]])
    err = max(np.mean([e for _, e in vals[nsmi.NS_FP64]]), 0.1)
    _say("logZ fp64", z64, "mixed", zmx)
    assert abs(z64.mean() - zmx.mean()) < 3 * err


@pytest.mark.parametrize("name", ["tiny", "paper"])
def test_theta_from_u_matches_oracle_prior_transform(name):
    """Unit-cube points to physical parameters (Tab. 1 transforms) on the
    GPU against the oracle's prior transform, including the cube's corners."""
    nsmi = _nsmi()
    ev, spec, data, _ = both_sides(WORKLOADS[name]())
    rng = np.random.default_rng(17)
    u = rng.random((257, spec.ndim))
    u[0] = 0.0
    u[1] = 1.0
    with nsmi.Context([spec], [data], n_live=8, num_delete=4, naccept=5, maxmcmc=10,
                      walk0=5) as ctx:
        ut = torch.tensor(u, device="cuda")
        th = torch.empty((len(u), 11), dtype=torch.float64, device="cuda")
        ctx.theta_from_u(0, ut, th)
        torch.cuda.synchronize()
        got = th.cpu().numpy()
        with pytest.raises(nsmi.NSError):
            ctx.theta_from_u(1, ut, th)
    want = np.array([oracle.prior_transform(ev, x) for x in u])
    err = np.abs(got - want) / np.maximum(1.0, np.abs(want))
    _say(f"theta_from_u {name}: max rel err {err.max():.2e}")
    assert err.max() <= 1e-12
