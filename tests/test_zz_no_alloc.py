"""The allocation-free entry point ns_signal_noalloc (for callers that cannot
call hipMalloc) against ns_signal: the same strain bit for bit, on two calls
in a row, the second with a smaller event; sizes beyond its scratch limit
are refused."""
import numpy as np
import pytest

from paper_2509_04336_amd import inputs

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")


def _nsmi():
    from paper_2509_04336_amd import nsmi
    return nsmi


def test_signal_noalloc_equals_signal_on_consecutive_calls():
    nsmi = _nsmi()
    big = inputs.paper_event(duration=16.0, f_hi=1024.0)     # 16 065 bins, 3 detectors
    small = inputs.tiny_event()                             # 945 bins, 1 detector
    th_big = np.array(big.theta_inj, dtype=np.float64)
    th_small = np.array(small.theta_inj, dtype=np.float64)
    print("noalloc: big event", big.n_bins, "bins x", big.n_det, flush=True)
    a1 = nsmi.signal_noalloc(big, th_big)
    print("noalloc: small event", small.n_bins, "bins x", small.n_det, flush=True)
    a2 = nsmi.signal_noalloc(small, th_small)
    b1 = nsmi.signal(big, th_big)
    b2 = nsmi.signal(small, th_small)
    assert a1.shape == b1.shape and a2.shape == b2.shape
    assert np.array_equal(a1, b1)
    assert np.array_equal(a2, b2)
    assert np.abs(a1).max() > 0 and np.abs(a2).max() > 0
    # a third call with the big event again: nothing of the small call remains
    assert np.array_equal(nsmi.signal_noalloc(big, th_big), b1)


def test_signal_noalloc_refuses_sizes_beyond_its_scratch():
    nsmi = _nsmi()
    spec = inputs.paper_event(duration=128.0, f_hi=1024.0)  # 128 513 bins > 65 536
    assert spec.n_bins > 65536
    with pytest.raises(nsmi.NSError) as ei:
        nsmi.signal_noalloc(spec, np.array(spec.theta_inj, dtype=np.float64))
    assert ei.value.status == nsmi.NS_EINVAL
    assert "65536" in str(ei.value)
