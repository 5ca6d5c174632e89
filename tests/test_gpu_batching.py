"""Multi-event batching on the GPU: several events of uneven length in one
context, walked by the same launches with their own tuned walk lengths.

* Each event matches a single-event oracle run with the same event index
  (chain ids and Philox streams carry the event index): live sets, dead
  points, counts and walk lengths agree exactly.
* Replaying each iteration as a captured hipGraph gives bit-identical results
  to eager launches (several replays, with host reads in between).
* The autotuner leaves the sampler state unchanged, and results do not depend
  on the launch shape it picks.
"""
import numpy as np
import pytest

import oracle
from helpers import WORKLOADS, both_sides
from paper_2509_04336_amd import inputs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _say(*a):
    print(*a, flush=True)


def _nsmi():
    from paper_2509_04336_amd import nsmi
    return nsmi


def _events():
    out = []
    for e, (T, fhi) in enumerate(((4.0, 512.0), (8.0, 256.0), (4.0, 300.0))):
        u, snr = inputs.multi_event_theta(e)
        spec = inputs.paper_event(duration=T, f_hi=fhi, seed=0, event=e, snr=snr)
        ev0 = oracle.event_from_spec(spec)
        th = oracle.prior_transform(ev0, u)
        import dataclasses
        spec = dataclasses.replace(spec, theta_inj=th, fixed_theta=th.copy())
        out.append(both_sides(spec))
    return out


def test_multi_event_parity_per_event():
    nsmi = _nsmi()
    evs = _events()
    n_live, k, seed = 60, 30, 5
    specs = [s for _, s, _, _ in evs]
    datas = [d for _, _, d, _ in evs]
    _say("bins per event", [s.n_bins for s in specs])
    ctx = nsmi.Context(specs, datas, n_live=n_live, num_delete=k, naccept=20, maxmcmc=5000,
                       walk0=8, seed=seed)
    nss = [oracle.NS(ev, n_live=n_live, naccept=20, maxmcmc=5000, walk0=8, seed=seed, event_id=e)
           for e, (ev, _, _, _) in enumerate(evs)]
    for e, ns in enumerate(nss):
        uo, Lo = ns.live()
        ug, Lg = ctx.live(e)
        assert np.array_equal(ug, uo)
        ctx.set_live(e, uo, Lo)
    for it in range(3):
        ctx.step()
        for ns in nss:
            ns.step(k)
        Ws = []
        for e, ns in enumerate(nss):
            ug, Lg = ctx.live(e)
            uo, Lo = ns.live()
            assert np.abs(ug - uo).max() <= 1e-12, (e, it)
            assert np.abs(Lg - Lo).max() <= 1e-6
            eg = ctx.evidence(e)
            so = ns.stats()
            assert eg["W"] == ns.W and eg["last_calls"] == so["last_calls"]
            assert abs(eg["logZ"] - ns.evidence()["logZ"]) <= 1e-6
            Ws.append(eg["W"])
        _say("iteration", it, "walk lengths per event", Ws)
    ctx.close()


def _run(nsmi, spec, data, graph, steps, wpc=0, autotune=False):
    stream = torch.cuda.Stream()
    with nsmi.Context([spec], [data], n_live=100, num_delete=50, naccept=30, maxmcmc=5000,
                      walk0=20, seed=3, stream=stream, graph=graph) as ctx:
        if wpc:
            ctx.set_waves_per_chain(wpc)
        chosen = None
        if autotune:
            before = ctx.live(), ctx.evidence()
            chosen = ctx.autotune(None, 32)
            after = ctx.live(), ctx.evidence()
            assert np.array_equal(before[0][0], after[0][0]) and np.array_equal(before[0][1], after[0][1])
            assert before[1] == after[1]
        out = []
        for i in range(steps):
            ctx.step()
            if i % 2 == 1:  # host reads between replays
                out.append(ctx.evidence()["logZ"])
        stream.synchronize()
        u, L = ctx.live()
        return u, L, ctx.evidence(), out, chosen


def test_graph_replays_match_eager_launches():
    nsmi = _nsmi()
    _, spec, data, _ = both_sides(inputs.tiny_event())
    ue, Le, ee, oe = _run(nsmi, spec, data, False, 8)[:4]
    ug, Lg, eg, og = _run(nsmi, spec, data, True, 8)[:4]
    assert np.array_equal(ue, ug) and np.array_equal(Le, Lg)
    assert oe == og and ee == eg


def test_autotune_is_side_effect_free_and_shape_independent():
    nsmi = _nsmi()
    _, spec, data, _ = both_sides(inputs.tiny_event())
    u1, L1, e1, _, chosen = _run(nsmi, spec, data, False, 6, autotune=True)
    _say("autotuner chose", chosen, "waves per chain")
    assert chosen in (1, 2, 4, 6, 8)
    for w in (1, 8):
        u2, L2, e2, _, _ = _run(nsmi, spec, data, False, 6, wpc=w)
        assert np.array_equal(u1, u2) and np.array_equal(L1, L2)
        e1c = dict(e1); e2c = dict(e2)
        e1c.pop("n_spec_discarded"); e2c.pop("n_spec_discarded")
        assert e1c == e2c


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_launch_shapes_give_identical_bits_paper_scale(precision):
    """Three detectors, 63 rows: the walk's log-likelihoods do not depend on
    how many waves share a chain (one wave per candidate, or candidate pairs
    on wave pairs splitting the rows), and equal those of the one-wave-per-
    point likelihood kernel bit for bit, in both precisions."""
    nsmi = _nsmi()
    _, spec, data, _ = both_sides(WORKLOADS["paper"]())
    prec = nsmi.NS_MIXED if precision == "mixed" else nsmi.NS_FP64
    res = {}
    for w in (1, 2, 4, 6, 8):
        _say("paper-scale walk with", w, "waves per chain,", precision)
        with nsmi.Context([spec], [data], n_live=200, num_delete=100, naccept=20, maxmcmc=5000,
                          walk0=12, seed=21, precision=prec) as ctx:
            ctx.set_waves_per_chain(w)
            for _ in range(2):
                ctx.step(100, 12)
            u, L = ctx.live()
            ev = ctx.evidence()
            ut = torch.tensor(u, device="cuda")
            out = torch.empty(len(L), dtype=torch.float64, device="cuda")
            ctx.loglike_batch_u(0, ut, out, prec)
            torch.cuda.synchronize()
            assert np.array_equal(out.cpu().numpy(), L)
            res[w] = (u, L, ev["logZ"], ev["n_calls"])
    u1, L1, z1, c1 = res[1]
    for w, (u, L, z, c) in res.items():
        assert np.array_equal(u, u1) and np.array_equal(L, L1), w
        assert z == z1 and c == c1, w
