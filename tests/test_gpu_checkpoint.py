"""Checkpoint and resume: a context restored from a checkpoint continues
exactly as the checkpointed run (the random numbers are keyed by the batch
index, so nothing else is needed); a bad checkpoint is refused without
changing the context."""
import dataclasses

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


# Byte offsets in a checkpoint: a 96-byte header, then the first event's
# state (ten doubles, ten int64 counters, eight int32 fields).
_HDR = 96
_OFF_LOGX, _OFF_BATCH, _OFF_W, _OFF_CONV = _HDR + 8, _HDR + 80 + 5 * 8, _HDR + 160, _HDR + 176


def _patched(ck, off, fmt, value):
    import struct
    b = bytearray(ck)
    struct.pack_into(fmt, b, off, value)
    return bytes(b)


def test_checkpoints_with_impossible_states_or_other_data_are_refused():
    import struct
    nsmi = _nsmi()
    _, spec, data, _ = both_sides(inputs.tiny_event())
    with _ctx(nsmi, spec, data, "walk") as a:
        for _ in range(2):
            a.step()
        ck = a.checkpoint()
        e = a.evidence()
    # the offsets read back what the context reports
    assert struct.unpack_from("<i", ck, _OFF_W)[0] == e["W"]
    assert struct.unpack_from("<q", ck, _OFF_BATCH)[0] == e["batch"]
    assert struct.unpack_from("<d", ck, _OFF_LOGX)[0] == e["logX"]
    bad = [
        _patched(ck, _OFF_W, "<i", 5001),            # walk length above maxmcmc
        _patched(ck, _OFF_W, "<i", 0),
        _patched(ck, _OFF_CONV, "<i", 7),            # flag not 0 or 1
        _patched(ck, _OFF_LOGX, "<d", 0.5),          # log X > 0
        _patched(ck, _OFF_LOGX, "<d", float("nan")),
        _patched(ck, _OFF_BATCH, "<q", -3),
    ]
    # the same shape and configuration on other data (a louder injection)
    spec2 = dataclasses.replace(spec, target_snr=25.0)
    _, spec2, data2, _ = both_sides(spec2)
    with _ctx(nsmi, spec, data, "walk") as same, _ctx(nsmi, spec2, data2, "walk") as other:
        for b in bad:
            before = _state(same)
            with pytest.raises(nsmi.NSError):
                same.restore(b)
            _same(_state(same), before)
        before = _state(other)
        with pytest.raises(nsmi.NSError) as ei:
            other.restore(ck)
        assert "other event data" in str(ei.value)
        _same(_state(other), before)
        same.restore(ck)  # the untouched checkpoint still loads
        assert same.evidence() == e
        same.step()
