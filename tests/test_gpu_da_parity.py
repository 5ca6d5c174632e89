"""Chain-level parity of the walks whose decisions depend on reduced
precision, against the oracle's FP64 chains, and the GPU Adam against the
oracle's.

* Delayed-acceptance walk with a non-constant screen (`walk_da_kernel` vs
  `or_walk_da`): the GPU screen is a BF16 network (FP32 accumulation), the
  oracle's the same parameters in FP64, so a screen decision of the two
  sides can differ only where |log U - log(pi ratio)| is below the screen
  error.  The oracle records, per chain, the smallest such gap over all of
  its screen decisions and the smallest |L' - L*| over its exact tests.  A
  chain whose gaps exceed the screen error bound (twice the largest
  |s_gpu - s_oracle| measured on the same network, over the temperature, and
  a safety factor of 2) and the FP64 likelihood tolerance takes the same
  decisions on both sides: its end point, log-likelihood and counts (accepts,
  exact calls, out-of-cube steps) must be equal.  Chains with a near tie are
  excluded and counted; most chains must be comparable.
* Mixed-precision walk: the GPU's mixed likelihood differs from the FP64
  oracle by up to 1e-3 per call; chains whose exact tests all have
  |L' - L*| > 1e-3 (gaps from the oracle's delayed-acceptance walk with a
  constant screen, which is the plain walk) must match exactly.
* Adam: training on pairs that all equal one point gives the same gradient
  at every step (the BF16 working weights do not move at a learning rate of
  1e-6); T steps of the GPU Adam must then equal T steps of or_adam_step fed
  with that gradient and the same learning-rate schedule.
"""
import math

import numpy as np
import pytest

import oracle
from helpers import WORKLOADS, both_sides

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _say(*a):
    print(*a, flush=True)


def _nsmi():
    from paper_2509_04336_amd import nsmi
    return nsmi


def _bf16_exact(p):
    """Round float values to the nearest BF16 (ties to even), as float64."""
    a = np.ascontiguousarray(np.asarray(p, dtype=np.float32))
    b = a.view(np.uint32).astype(np.uint64)
    b = (b + 0x7FFF + ((b >> 16) & 1)) & 0xFFFF0000
    return b.astype(np.uint32).view(np.float32).astype(np.float64)


def _screen_params(seed, w1_scale=6.0):
    """A random network whose output varies over the unit cube by about ten
    times its BF16 evaluation error (the first layer is scaled up so the
    inputs in [0, 1] move it)."""
    rng = np.random.default_rng(seed)
    p = np.zeros(oracle.mlp_num_params())
    W1, b1, W2, b2, W3, b3, W4, b4 = oracle.mlp_unpack(p)
    for W, fan, sc in ((W1, 11, w1_scale), (W2, 256, 1.0), (W3, 256, 1.0), (W4, 256, 1.0)):
        W[...] = rng.uniform(-1, 1, W.shape) * 1.5 * sc / np.sqrt(fan)
    for b in (b1, b2, b3, b4):
        b[...] = rng.uniform(-0.2, 0.2, b.shape)
    return _bf16_exact(p)


def _screen_error(ctx, screen, ndim, rng, n=4096, live_u=None):
    """Largest |s_gpu - s_oracle| over uniform points of the cube (and the
    live points, if given)."""
    u = rng.random((n, ndim))
    if live_u is not None:
        u = np.vstack([u, live_u])
    out = torch.empty(len(u), dtype=torch.float64, device="cuda")
    ctx.surrogate_predict(torch.tensor(u, device="cuda"), out)
    got = out.cpu().numpy()
    want = screen.predict(ndim, u)
    return float(np.abs(got - want).max())


def _da_case(name, n_live, k, W, seeds, sigma, temp, floor, min_frac):
    nsmi = _nsmi()
    ev, spec, data, _ = both_sides(WORKLOADS[name]())
    d = spec.ndim
    p = _screen_params(31)
    rng = np.random.default_rng(5)
    total, comparable, saved_total = 0, 0, 0
    for seed in seeds:
        ns = oracle.NS(ev, n_live=n_live, naccept=20, maxmcmc=5000, walk0=W, seed=seed)
        ctx = nsmi.Context([spec], [data], n_live=n_live, num_delete=k, naccept=20, maxmcmc=5000,
                           walk0=W, seed=seed)
        uo, Lo = ns.live()
        ctx.set_live(0, uo, Lo)
        # the first selection deletes the k lowest: L* is the k-th smallest
        Lstar = float(np.sort(Lo)[k - 1])
        margin = Lstar  # sigmoid argument (s - L* + margin) / temp = s / temp
        screen = oracle.Screen(p, in_mean=np.zeros(d), in_sd=np.ones(d), mu=0.0, sigma=sigma,
                               margin=margin, temp=temp, floor=floor)
        ctx.surrogate_init(seed=0, max_rows=4096)
        ctx.surrogate_set_params(p)
        ctx.surrogate_set_norm(0.0, sigma)
        ctx.surrogate_set_input_norm(np.zeros(d), np.ones(d))
        ctx.surrogate_attach(margin, temp, floor)
        eps_s = _screen_error(ctx, screen, d, rng, live_u=uo)
        thr = 2.0 * (2.0 * eps_s / temp)
        ns.set_screen(screen)
        ns.step(k, W)
        ctx.step(k, W)
        assert abs(ns.last_Lstar - Lstar) == 0.0
        ug, Lg = ctx.live()
        uo2, Lo2 = ns.live()
        # survivors (rows 0 .. n-k-1) are the same rows on both sides
        assert np.array_equal(ug[: n_live - k], uo2[: n_live - k])
        gs, gl = ns.last_gaps()
        co = ns.last_chains()
        cg = ctx.chain_stats()
        assert cg.shape == (k, 4) and co.shape == (k, 3)
        ok = (gs > thr) & (gl > 1e-5)
        rows = n_live - k + np.nonzero(ok)[0]
        du = np.abs(ug[rows] - uo2[rows]).max() if len(rows) else 0.0
        dL = np.abs(Lg[rows] - Lo2[rows]).max() if len(rows) else 0.0
        assert du <= 1e-12, du
        assert dL <= 1e-6, dL
        assert np.array_equal(cg[ok, :3], co[ok]), np.nonzero((cg[:, :3] != co).any(axis=1) & ok)
        saved_g = W - cg[:, 1] - cg[:, 2]
        saved_o = W - co[:, 1] - co[:, 2]
        assert np.array_equal(saved_g[ok], saved_o[ok])
        if ok.all():
            eg = ctx.evidence()
            assert eg["n_calls_saved"] == ns.n_saved
        total += k
        comparable += int(ok.sum())
        saved_total += int(saved_o[ok].sum())
        _say(f"DA {name} seed {seed}: screen error {eps_s:.2e}, gap threshold {thr:.2e}, "
             f"comparable chains {int(ok.sum())}/{k}, accepts {int(co[:, 0].sum())}, "
             f"calls {int(co[:, 1].sum())}, saved {int(saved_o.sum())}")
        ctx.close()
    assert saved_total > 0, "the screen must reject some proposals in stage 1"
    assert comparable >= min_frac * total, (comparable, total)


# Screen settings: the more a screen varies relative to its BF16 error, and
# the more decisions a chain takes, the more chains have a near tie; these
# keep about half of the chains comparable (estimated with the oracle and a
# BF16 emulation of the network) while the screen still rejects proposals.

def test_delayed_acceptance_walk_matches_oracle_tiny():
    _da_case("tiny", 100, 50, 24, seeds=(1, 2, 3), sigma=2.0, temp=2.0, floor=0.0, min_frac=0.4)


def test_delayed_acceptance_walk_matches_oracle_tiny_long_walk_with_floor():
    # 120 steps: several candidate rounds and draw windows per chain
    _da_case("tiny", 100, 50, 120, seeds=(4, 5), sigma=0.5, temp=2.0, floor=0.1, min_frac=0.3)


def test_delayed_acceptance_walk_matches_oracle_paper_scale():
    # 11-D, three detectors, 4017 bins: the exact FP64 evaluation path of the
    # delayed-acceptance kernel
    _da_case("paper", 64, 32, 24, seeds=(6, 7), sigma=1.0, temp=2.0, floor=0.05, min_frac=0.4)


def _mixed_case(name, n_live, k, W, seeds, min_frac):
    nsmi = _nsmi()
    ev, spec, data, _ = both_sides(WORKLOADS[name]())
    total, comparable = 0, 0
    for seed in seeds:
        ns = oracle.NS(ev, n_live=n_live, naccept=20, maxmcmc=5000, walk0=W, seed=seed)
        ns.set_screen(oracle.Screen(None, const_s=1e3))  # the plain walk, with its gaps
        ctx = nsmi.Context([spec], [data], n_live=n_live, num_delete=k, naccept=20, maxmcmc=5000,
                           walk0=W, seed=seed, precision=nsmi.NS_MIXED)
        uo, Lo = ns.live()
        ctx.set_live(0, uo, Lo)
        ns.step(k, W)
        ctx.step(k, W)
        ug, Lg = ctx.live()
        uo2, Lo2 = ns.live()
        assert np.array_equal(ug[: n_live - k], uo2[: n_live - k])
        _, gl = ns.last_gaps()
        co = ns.last_chains()
        cg = ctx.chain_stats()
        ok = gl > 1e-3
        rows = n_live - k + np.nonzero(ok)[0]
        if len(rows):
            assert np.abs(ug[rows] - uo2[rows]).max() <= 1e-12
            assert np.abs(Lg[rows] - Lo2[rows]).max() <= 1e-3
        assert np.array_equal(cg[ok, :3], co[ok])
        if ok.all():
            eg = ctx.evidence()
            st = ns.stats()
            assert eg["last_accept"] == st["last_acc"] and eg["last_calls"] == st["last_calls"]
        total += k
        comparable += int(ok.sum())
        _say(f"mixed walk {name} seed {seed}: comparable chains {int(ok.sum())}/{k}, "
             f"accepts {int(co[:, 0].sum())}, calls {int(co[:, 1].sum())}")
        ctx.close()
    assert comparable >= min_frac * total, (comparable, total)


def test_mixed_precision_walk_chains_match_oracle_tiny():
    _mixed_case("tiny", 100, 50, 60, seeds=(1, 2), min_frac=0.8)


def test_mixed_precision_walk_chains_match_oracle_paper_scale():
    _mixed_case("paper", 64, 32, 40, seeds=(3,), min_frac=0.8)


@pytest.mark.parametrize("n,batch", [(256, 64), (1024, 1024), (1000, 1000)])
def test_gpu_adam_matches_oracle_adam(n, batch):
    # batch 64: one launch per gradient reduction, then Adam; batch 1024: the
    # weight gradients split over the batch, their partial sums and the bias
    # sums reduced inside Adam's launch; batch 1000: the same with 24 padding
    # rows in the last forward product's output-layer epilogue
    nsmi = _nsmi()
    _, spec, data, _ = both_sides(WORKLOADS["tiny"]())
    T, lr = 12, 1e-6
    u = np.full((n, 4), 0.5)       # input mean 0.5, spread 0: standardised input 0
    L = np.zeros(n)                # target mean 0, spread 0: normalised target 0
    with nsmi.Context([spec], [data], n_live=8, num_delete=4, naccept=5, maxmcmc=10,
                      walk0=5) as ctx:
        ctx.surrogate_init(seed=3, max_rows=max(512, n))
        # a network with a non-zero output (the initial output layer is zero)
        ctx.surrogate_set_params(_screen_params(3, w1_scale=1.0))
        p0 = ctx.surrogate_get_params().astype(np.float64)
        # the normalisation training will derive from these pairs
        ctx.surrogate_set_norm(0.0, 1.0)
        ctx.surrogate_set_input_norm(np.full(4, 0.5), np.ones(4))
        ut, Lt = torch.tensor(u, device="cuda"), torch.tensor(L, device="cuda")
        _, g = ctx.surrogate_loss_grad(ut, Lt)
        ctx.surrogate_train(ut, Lt, steps=T, batch=batch, lr=lr)
        assert ctx.surrogate_get_norm()[:2] == (0.0, 1.0)
        m_in, sd_in = ctx.surrogate_get_input_norm()
        assert np.all(m_in == 0.5) and np.all(sd_in == 1.0)
        pT = ctx.surrogate_get_params().astype(np.float64)
    g = g.astype(np.float64)
    # the oracle's Adam on the same gradient and learning-rate schedule
    p, m, v = p0.copy(), np.zeros_like(p0), np.zeros_like(p0)
    for t in range(1, T + 1):
        frac = (t - 1) / (T - 1)
        lr_t = float(np.float32(lr * (0.05 + 0.95 * 0.5 * (1.0 + math.cos(math.pi * frac)))))
        oracle.adam_step(p, g, m, v, t, lr=lr_t)
    dg, do = pT - p0, p - p0
    rel = np.linalg.norm(dg - do) / np.linalg.norm(do)
    cos = float(dg @ do / (np.linalg.norm(dg) * np.linalg.norm(do)))
    W1 = oracle.mlp_unpack(do)[0]
    _say(f"Adam over {T} steps: |dp| {np.linalg.norm(do):.3e}, rel-L2 {rel:.2e}, cosine {cos:.8f}, "
         f"max |d| {np.abs(dg - do).max():.2e}")
    assert np.all(W1 == 0.0) and np.all(oracle.mlp_unpack(dg)[0] == 0.0)  # zero input: no W1 step
    assert rel <= 2e-3 and cos >= 0.99999
