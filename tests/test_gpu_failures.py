"""Failure handling forced from the host: a threshold above every proposal,
a corrupted autotuner cache, and run-twice bitwise determinism (with
counter-based random numbers and fixed-order reductions, any difference
between two identical runs is a race)."""
import numpy as np
import pytest

from helpers import WORKLOADS, both_sides
from paper_2509_04336_amd import inputs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _nsmi():
    from paper_2509_04336_amd import nsmi
    return nsmi


@pytest.mark.parametrize("inner", ["walk", "hrss"])
def test_threshold_above_every_proposal_returns_the_start_points(inner):
    # live log-likelihoods far above anything the data allow (distinct, so
    # survivors above L* exist): no proposal can pass, every chain returns
    # the survivor it started from, and the walk length goes to the cap
    nsmi = _nsmi()
    _, spec, data, _ = both_sides(inputs.tiny_event())
    n, k, cap = 60, 30, 40
    with nsmi.Context([spec], [data], n_live=n, num_delete=k, naccept=10, maxmcmc=cap, walk0=8,
                      seed=41, inner=inner) as ctx:
        assert ctx.evidence()["walk_capped"] == 0
        u0, _ = ctx.live()
        L0 = 1e10 + np.arange(n, dtype=np.float64)
        ctx.set_live(0, u0, L0)
        ctx.step()
        e = ctx.evidence()
        assert e["last_accept"] == 0
        assert e["W"] == cap
        assert e["walk_capped"] == 1  # the stuck-walk guard counts capped batches
        assert e["last_Lstar"] == L0[k - 1]
        u1, L1 = ctx.live()
        survivors = {tuple(r) for r in u0[k:]}
        for r, l in zip(u1, L1):
            assert tuple(r) in survivors
            i = np.flatnonzero((u0 == r).all(axis=1))[0]
            assert l == L0[i]
        ctx.step()  # still nothing passes: the guard keeps counting
        e = ctx.evidence()
        assert e["last_accept"] == 0 and e["W"] == cap and e["walk_capped"] == 2


def test_corrupted_autotuner_cache_falls_back_to_tuning(tmp_path):
    nsmi = _nsmi()
    _, spec, data, _ = both_sides(inputs.tiny_event())
    path = tmp_path / "tune.txt"

    def tune():
        with nsmi.Context([spec], [data], n_live=100, num_delete=50, naccept=20, maxmcmc=5000,
                          walk0=10, seed=42) as ctx:
            return ctx.autotune(str(path), 16)

    first = tune()
    assert first in (1, 2, 4, 6, 8)
    key = path.read_text().splitlines()[-1].rsplit(" | ", 1)[0]
    # garbage, a wrong key, and values the kernel does not take: all ignored
    path.write_text("\x00\xffgarbage\n" + key + " | 7\n" + key + " | abc\n" + key + "\n"
                    + "other key | 4\n" + key + " | 999\n")
    again = tune()
    assert again in (1, 2, 4, 6, 8)
    assert path.read_text().splitlines()[-1] == f"{key} | {again}"  # re-tuned and appended
    # a valid entry is read back (including 6) without re-tuning
    path.write_text(f"{key} | 6\n")
    assert tune() == 6
    assert path.read_text() == f"{key} | 6\n"


@pytest.mark.parametrize("inner,precision", [("walk", "fp64"), ("walk", "mixed"), ("hrss", "fp64")])
def test_two_identical_runs_give_identical_bits_paper_scale(inner, precision):
    nsmi = _nsmi()
    _, spec, data, _ = both_sides(WORKLOADS["paper"]())
    prec = nsmi.NS_MIXED if precision == "mixed" else nsmi.NS_FP64

    def run():
        with nsmi.Context([spec], [data], n_live=1000, num_delete=500, naccept=60, maxmcmc=5000,
                          walk0=100, seed=43, precision=prec, inner=inner) as ctx:
            for _ in range(3):
                ctx.step()
            u, L = ctx.live()
            return u, L, ctx.dead(), ctx.evidence()

    a, b = run(), run()
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    for x, y in zip(a[2], b[2]):
        assert np.array_equal(x, y)
    assert a[3] == b[3]
    print(inner, precision, "log Z after 3 batches", a[3]["logZ"], flush=True)
