"""Values the paper prints, checked against the inputs module and the
oracle's volume accounting."""
import json
import math
import os

import numpy as np

import oracle
from paper_2509_04336_amd import inputs

G = os.path.join(os.path.dirname(__file__), "golden")


def _load(name):
    with open(os.path.join(G, name)) as f:
        return json.load(f)


def test_injection_tables_match_paper():
    t = _load("injection_tables.json")
    np.testing.assert_array_equal(inputs.TABLE2_INJECTION, np.array(t["table2_4s"]))
    np.testing.assert_array_equal(inputs.TABLE4_INJECTION, np.array(t["table4_8s"]))


def test_live_point_matching_rule():
    g = _load("volume_shrinkage.json")
    n, k, ncpu = g["n_gpu"], g["k"], g["n_cpu"]
    # exact per-batch shrinkage, as the oracle accounts it
    ev, _, _ = oracle.build_event(inputs.toy_event(2, 0.1))
    ns = oracle.NS(ev, n_live=n, naccept=5, maxmcmc=10, seed=0)
    ns.step(k, walk=1)
    shrink = -ns.evidence()["logX"]
    assert abs(shrink - math.log(n / (n - k))) < 1.0 / n
    assert abs(math.log(2) - g["ln2"]) < 1e-15
    # k / n_cpu = ln(n / (n - k)) with k = n/2 -> n = 2 ln 2 n_cpu ~ 1.39 n_cpu
    assert abs(2 * math.log(2) * ncpu / n - 1.0) < 0.01
    assert abs(round(2 * math.log(2), 1) - g["ratio_printed"]) < 1e-12


def test_logz_reference_reproduces_from_the_oracle():
    """tests/golden/logz_ref.json holds oracle-only evidence runs of the 4-D
    workload (written by make_logz_ref.py); seed 0 of the 945-bin event is
    re-run here and must give the stored value (the same arithmetic, up to
    the reduction order of the threads)."""
    g = _load("logz_ref.json")
    run0 = g["tiny"]["runs"][0]
    ev, _, _ = oracle.build_event(inputs.tiny_event())
    s = inputs.TINY_SAMPLER
    ns = oracle.NS(ev, n_live=s.n_live, naccept=s.naccept, maxmcmc=s.maxmcmc, walk0=s.walk0,
                   seed=run0["seed"])
    e = ns.run(s.num_delete, s.term_kind, s.term_thr)
    assert abs(e["logZ"] - run0["logZ"]) < 1e-9
    assert ns.batch == run0["batches"]
    z = np.array([r["logZ"] for r in g["tiny"]["runs"]])
    assert abs(z.mean() - g["tiny"]["logZ_ref"]) < 1e-12
