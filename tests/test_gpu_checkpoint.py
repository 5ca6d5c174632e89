"""Checkpoint and resume: a context restored from a checkpoint continues
exactly as the checkpointed run (the random numbers are keyed by the batch
index, so nothing else is needed); a bad checkpoint is refused without
changing the context."""
import numpy as np
import pytest

from helpers import both_sides
from paper_2509_04336_amd import inputs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _nsmi():
    from paper_2509_04336_amd import nsmi
    return nsmi


def _ctx(nsmi, spec, data, inner, seed=21, graph=False):
    # captured iterations need a stream of their own (the null stream cannot be captured)
    stream = torch.cuda.Stream() if graph else None
    return nsmi.Context([spec], [data], n_live=100, num_delete=50, naccept=20, maxmcmc=5000,
                        walk0=10, term_kind=1, term_thr=1e-3, seed=seed, inner=inner, graph=graph,
                        stream=stream)


def _state(ctx):
    u, L = ctx.live()
    du, dL, dw, dn = ctx.dead()
    return u, L, du, dL, dw, dn, ctx.evidence()


def _same(a, b):
    for x, y in zip(a[:6], b[:6]):
        assert np.array_equal(x, y)
    assert a[6] == b[6]


@pytest.mark.parametrize("inner", ["walk", "hrss"])
def test_resumed_context_continues_bit_for_bit(inner):
    nsmi = _nsmi()
    _, spec, data, _ = both_sides(inputs.tiny_event())
    with _ctx(nsmi, spec, data, inner) as a:
        for _ in range(4):
            a.step()
        ck = a.checkpoint()
        for _ in range(4):
            a.step()
        want = _state(a)
    print(inner, "checkpoint bytes", len(ck), "dead after 8 batches", len(want[3]), flush=True)
    with _ctx(nsmi, spec, data, inner, graph=True) as b:
        b.restore(ck)
        for _ in range(4):
            b.step()
        _same(_state(b), want)


def test_restore_rolls_a_context_back():
    nsmi = _nsmi()
    _, spec, data, _ = both_sides(inputs.tiny_event())
    with _ctx(nsmi, spec, data, "walk") as a:
        for _ in range(3):
            a.step()
        ck = a.checkpoint()
        at_ck = _state(a)
        for _ in range(3):
            a.step()
        first = _state(a)
        a.restore(ck)
        _same(_state(a), at_ck)
        for _ in range(3):
            a.step()
        _same(_state(a), first)


def test_bad_checkpoints_are_refused_without_change():
    nsmi = _nsmi()
    _, spec, data, _ = both_sides(inputs.tiny_event())
    with _ctx(nsmi, spec, data, "walk") as a:
        for _ in range(2):
            a.step()
        ck = a.checkpoint()
    with _ctx(nsmi, spec, data, "walk", seed=22) as other, _ctx(nsmi, spec, data, "hrss") as hr:
        for bad, ctx in ((ck, other), (ck, hr), (ck[:-8], other), (b"X" + ck[1:], other),
                         (ck + b"\0" * 8, other), (ck[:40], other)):
            before = _state(ctx)
            with pytest.raises(nsmi.NSError):
                ctx.restore(bad)
            _same(_state(ctx), before)
        other.step()  # still usable
