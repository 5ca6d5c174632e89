"""Percentile-percentile coverage of the 4-D event (intrinsic parameters,
extrinsic ones fixed, seeded noise, SNR 20) with the GPU sampler or with the
CPU oracle sampler on the same injections, for comparing the two samplers'
posteriors statistically end to end (not collected by pytest: the oracle
takes about half an hour for 100 injections).

    python tests/pp_gpu_vs_oracle.py gpu|oracle N n_live num_delete naccept
"""
import dataclasses
import os
import sys
import time
sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
import numpy as np
from scipy import stats
from paper_2509_04336_amd import inputs
which = sys.argv[1]
N = int(sys.argv[2]); n_live = int(sys.argv[3]); k = int(sys.argv[4]); na = int(sys.argv[5])
base = inputs.tiny_event()
rng = np.random.default_rng([0, 9191])
u_inj = rng.random((N, 4))
lo, hi = base.prior_lo[:4], base.prior_hi[:4]
th_all = lo + u_inj * (hi - lo)   # the tiny prior is uniform in all four
if which == 'gpu':
    import torch
    from paper_2509_04336_amd import nsmi
    inject = nsmi.inject
else:
    import oracle
pct = np.zeros((N, 4)); t0 = time.time()
for i in range(N):
    th = base.theta_inj.copy(); th[:4] = th_all[i]
    spec = dataclasses.replace(base, theta_inj=th, fixed_theta=th.copy(),
                               noise=inputs.noise(0, 2000 + i, 1, base.psd, base.df))
    if which == 'gpu':
        data, _, fixed = nsmi.inject(spec)
        spec = dataclasses.replace(spec, fixed_theta=fixed)
        with nsmi.Context([spec], [data], n_live=n_live, num_delete=k, naccept=na, maxmcmc=5000,
                          walk0=100, term_kind=1, term_thr=1e-3, seed=i) as ctx:
            for _ in range(2000):
                if ctx.converged(): break
                ctx.step()
            ev = ctx.evidence(); ud, Ld, lwd, _ = ctx.dead(); ul, Ll = ctx.live()
        logX = ev['logX']
    else:
        ev0, th2, data = oracle.build_event(spec)
        ns = oracle.NS(ev0, n_live=n_live, naccept=na, maxmcmc=5000, walk0=100, seed=i)
        for _ in range(2000):
            if ns.evidence()['log_frac'] < np.log(1e-3): break
            ns.step(k)
        ud, Ld, lwd, _ = ns.dead(); ul, Ll = ns.live(); logX = ns.evidence()['logX']
    lw = np.concatenate([lwd + Ld, logX - np.log(n_live) + Ll]); w = np.exp(lw - lw.max()); w /= w.sum()
    us = np.concatenate([ud, ul])
    pct[i] = (w[:, None] * (us < u_inj[i][None, :])).sum(0)
ks = [stats.kstest(pct[:, j], 'uniform').pvalue for j in range(4)]
print(f"{which} N={N} n_live={n_live} k={k} naccept={na}: KS p " + " ".join(f"{v:.3g}" for v in ks)
      + f"; q-pct hist {np.histogram(pct[:, 1], bins=10, range=(0, 1))[0].tolist()}; {time.time() - t0:.0f} s", flush=True)
