"""Write logz_ref.json: the reference evidence of the 4-D workloads from the
FP64 oracle alone (nested sampling run to its termination rule, several
seeds), used as logZ_ref in the time-to-converged-evidence measurement.

    python tests/golden/make_logz_ref.py [--quick]

Workloads (the synthetic stand-ins of the paper's 4-D runs, Sec. 4.1):
  tiny: 4 s at 20-256 Hz (945 bins), zero noise, SNR 20, 100 live, 50
        deleted per batch, naccept 30, dlogZ < 0.1; seeds 0-9
  long: the same event at 8 s, 20-2048 Hz (16 225 bins); seeds 0-4
"""
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_2509_04336_amd import inputs  # noqa: E402


def run(spec, seeds):
    ev, _, _ = oracle.build_event(spec)
    s = inputs.TINY_SAMPLER
    out = []
    for seed in seeds:
        t0 = time.perf_counter()
        ns = oracle.NS(ev, n_live=s.n_live, naccept=s.naccept, maxmcmc=s.maxmcmc, walk0=s.walk0,
                       seed=seed)
        e = ns.run(s.num_delete, s.term_kind, s.term_thr)
        dt = time.perf_counter() - t0
        out.append({"seed": seed, "logZ": e["logZ"], "logZ_err": e["logZ_err"],
                    "batches": int(ns.batch), "calls": int(ns.stats()["calls"]),
                    "seconds": round(dt, 2)})
        print(f"seed {seed}: logZ {e['logZ']:.4f} +- {e['logZ_err']:.4f} ({dt:.1f} s)", flush=True)
    z = np.array([r["logZ"] for r in out])
    return {"logZ_ref": float(z.mean()), "sd_over_seeds": float(z.std(ddof=1)),
            "stderr": float(z.std(ddof=1) / np.sqrt(len(z))), "runs": out}


def main():
    quick = "--quick" in sys.argv
    oracle.build()
    res = {"generator": "tests/golden/make_logz_ref.py (FP64 oracle only)",
           "threads": oracle.num_threads(),
           "sampler": "100 live, 50 deleted per batch, naccept 30, maxmcmc 5000, dlogZ < 0.1"}
    res["tiny"] = dict(workload="4-D, 1 detector (F+ = 1), 4 s at 20-256 Hz, 945 bins, zero "
                                "noise, SNR 20", **run(inputs.tiny_event(), range(2 if quick else 10)))
    if not quick:
        res["long"] = dict(workload="the tiny event at 8 s, 20-2048 Hz, 16 225 bins",
                           **run(inputs.tiny_event(duration=8.0, f_hi=2048.0), range(5)))
    path = os.path.join(HERE, "logz_ref.json")
    with open(path, "w") as f:
        json.dump(res, f, indent=1)
    print("wrote", path)


if __name__ == "__main__":
    main()
