"""ctypes binding of libnsmi.so (the C ABI in include/nsmi.h).

Argument marshalling only: every step of the sampler runs in the library's
HIP kernels.  PyTorch supplies device memory and the stream; numpy arrays
carry host inputs.  Importing this module fails loudly when the library has
not been built (``python -m paper_2509_04336_amd.build``).
"""
from __future__ import annotations

import ctypes as C
import math
import os
from typing import Optional, Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libnsmi.so")

NS_OK, NS_EINVAL, NS_EHIP, NS_ENOMEM, NS_ESTATE, NS_ENONFINITE, NS_ENOTIMPL = 0, -1, -2, -3, -4, -5, -6
NS_FP64, NS_MIXED = 0, 1
NS_LIKE_GW, NS_LIKE_GAUSS, NS_LIKE_GW_RB = 0, 1, 2
NS_INNER_WALK, NS_INNER_HRSS = 0, 1

_STATUS = {0: "NS_OK", -1: "NS_EINVAL", -2: "NS_EHIP", -3: "NS_ENOMEM", -4: "NS_ESTATE",
           -5: "NS_ENONFINITE", -6: "NS_ENOTIMPL"}

D = C.POINTER(C.c_double)


class NSError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


class EventDesc(C.Structure):
    _fields_ = [("n_bins", C.c_int32), ("n_det", C.c_int32), ("ndim", C.c_int32),
                ("likelihood", C.c_int32), ("f_lo", C.c_double), ("df", C.c_double),
                ("data", D), ("psd", D), ("det_tensor", D), ("det_loc", D),
                ("fixed_antenna", D), ("prior_lo", D), ("prior_hi", D), ("fixed_theta", D),
                ("gmst", C.c_double), ("toy_sigma", C.c_double),
                ("rb_theta0", D), ("rb_edges", C.POINTER(C.c_int32)), ("rb_bins", C.c_int32),
                ("rb_pad", C.c_int32)]


class Config(C.Structure):
    _fields_ = [("n_live", C.c_int32), ("num_delete", C.c_int32), ("naccept", C.c_int32),
                ("maxmcmc", C.c_int32), ("walk0", C.c_int32), ("term_kind", C.c_int32),
                ("delay", C.c_double), ("term_thr", C.c_double), ("precision", C.c_int32),
                ("flags", C.c_int32), ("seed", C.c_uint64), ("stream", C.c_void_p)]


NS_FLAG_TIMING = 1
NS_FLAG_GRAPH = 2


class Timing(C.Structure):
    _fields_ = [("select_ms", C.c_double), ("walk_ms", C.c_double), ("finish_ms", C.c_double),
                ("launches", C.c_int64)]


class Evidence(C.Structure):
    _fields_ = [("logZ", C.c_double), ("logZ_dead", C.c_double), ("logZ_err", C.c_double),
                ("H", C.c_double), ("logX", C.c_double), ("dlogZ", C.c_double),
                ("log_frac", C.c_double), ("last_Lstar", C.c_double), ("n_dead", C.c_int64),
                ("n_calls", C.c_int64), ("n_accept", C.c_int64), ("n_oob", C.c_int64),
                ("n_steps", C.c_int64), ("n_calls_saved", C.c_int64), ("batch", C.c_int64),
                ("W", C.c_int32), ("converged", C.c_int32), ("last_accept", C.c_int64),
                ("last_calls", C.c_int64), ("n_spec_discarded", C.c_int64),
                ("walk_capped", C.c_int32), ("reserved", C.c_int32)]

    def to_dict(self) -> dict:
        return {name: getattr(self, name) for name, _ in self._fields_}


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_2509_04336_amd.build` (HIP, gfx950)")
        L = C.CDLL(LIB_PATH)
        V = C.c_void_p
        P = C.POINTER
        L.ns_init.argtypes = [P(V), P(Config), P(EventDesc), C.c_int32]
        L.ns_free.argtypes = [V]
        L.ns_free.restype = None
        L.ns_last_error.argtypes = [V]
        L.ns_last_error.restype = C.c_char_p
        L.ns_step.argtypes = [V, C.c_int32, C.c_int32]
        L.ns_get_chain_stats.argtypes = [V, C.c_int32, C.POINTER(C.c_int64), C.c_int32,
                                         C.POINTER(C.c_int32)]
        L.ns_loglike_batch.argtypes = [V, C.c_int32, V, C.c_int64, V, C.c_int32]
        L.ns_loglike_batch_u.argtypes = [V, C.c_int32, V, C.c_int64, V, C.c_int32]
        L.ns_evidence.argtypes = [V, C.c_int32, P(Evidence)]
        L.ns_get_live.argtypes = [V, C.c_int32, D, D]
        L.ns_set_live.argtypes = [V, C.c_int32, D, D]
        L.ns_get_dead.argtypes = [V, C.c_int32, C.c_int64, D, D, D, D, P(C.c_int64)]
        L.ns_checkpoint_size.argtypes = [V, P(C.c_int64)]
        L.ns_checkpoint.argtypes = [V, C.c_void_p, C.c_int64, P(C.c_int64)]
        L.ns_restore.argtypes = [V, C.c_void_p, C.c_int64]
        L.ns_signal.argtypes = [P(EventDesc), D, D]
        L.ns_signal_noalloc.argtypes = [P(EventDesc), D, D]
        L.ns_logz_replicates.argtypes = [V, C.c_int32, C.c_int32, C.c_uint64, V, V]
        L.ns_num_events.argtypes = [V]
        L.ns_num_events.restype = C.c_int32
        L.ns_version.restype = C.c_char_p
        L.ns_timing.argtypes = [V, P(Timing), C.c_int32]
        L.ns_set_waves_per_chain.argtypes = [V, C.c_int32]
        F = C.POINTER(C.c_float)
        L.ns_surrogate_init.argtypes = [V, C.c_uint64, C.c_int64]
        L.ns_surrogate_set_params.argtypes = [V, F, C.c_int64]
        L.ns_surrogate_get_params.argtypes = [V, F, C.c_int64]
        L.ns_surrogate_set_norm.argtypes = [V, C.c_double, C.c_double, C.c_double, C.c_double]
        L.ns_surrogate_get_norm.argtypes = [V, D, D, D, D]
        L.ns_surrogate_predict.argtypes = [V, V, C.c_int64, V]
        L.ns_surrogate_set_input_norm.argtypes = [V, D, D]
        L.ns_surrogate_get_input_norm.argtypes = [V, D, D]
        L.ns_surrogate_loss_grad.argtypes = [V, V, V, C.c_int64, F, D]
        L.ns_surrogate_train.argtypes = [V, V, V, C.c_int64, C.c_int32, C.c_int32, C.c_double,
                                         C.c_double, C.c_double, D]
        L.ns_harvest.argtypes = [V, C.c_int64]
        L.ns_theta_from_u.argtypes = [V, C.c_int32, V, C.c_int64, V]
        L.ns_set_inner.argtypes = [V, C.c_int32]
        L.ns_surrogate_attach.argtypes = [V, C.c_double, C.c_double, C.c_double]
        L.ns_autotune.argtypes = [V, C.c_char_p, C.c_int32, P(C.c_int32)]
        L.ns_surrogate_detach.argtypes = [V]
        L.ns_harvest_copy.argtypes = [V, V, V, C.c_int64, P(C.c_int64)]
        for f in ("ns_init", "ns_step", "ns_loglike_batch", "ns_loglike_batch_u", "ns_evidence",
                  "ns_get_live", "ns_set_live", "ns_get_dead", "ns_signal", "ns_timing",
                  "ns_checkpoint_size", "ns_checkpoint", "ns_restore",
                  "ns_set_waves_per_chain", "ns_surrogate_init", "ns_surrogate_set_params",
                  "ns_surrogate_get_params", "ns_surrogate_set_norm", "ns_surrogate_get_norm",
                  "ns_surrogate_predict", "ns_surrogate_loss_grad", "ns_surrogate_train",
                  "ns_harvest", "ns_harvest_copy", "ns_surrogate_attach", "ns_surrogate_detach", "ns_autotune",
                  "ns_surrogate_set_input_norm", "ns_surrogate_get_input_norm",
                  "ns_theta_from_u", "ns_set_inner", "ns_get_chain_stats", "ns_signal_noalloc", "ns_logz_replicates"):
            getattr(L, f).restype = C.c_int
        _lib = L
    return _lib


def version() -> str:
    return lib().ns_version().decode()


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def _ptr(a: Optional[np.ndarray]):
    return C.cast(None, D) if a is None else a.ctypes.data_as(D)


class _Desc:
    """An EventDesc plus the numpy arrays it points into (kept alive)."""

    def __init__(self, spec, data=None):
        if data is None:
            data = np.zeros((spec.n_det, spec.n_bins), np.complex128)
        data = np.asarray(data)
        if np.iscomplexobj(data):
            data = np.stack([data.real, data.imag], axis=-1)
        keep = dict(data=_f64(data).reshape(-1), psd=_f64(spec.psd).reshape(-1),
                    det_tensor=None if spec.det_tensor is None else _f64(spec.det_tensor).reshape(-1),
                    det_loc=None if spec.det_loc is None else _f64(spec.det_loc).reshape(-1),
                    fixed_antenna=None if spec.fixed_antenna is None else _f64(spec.fixed_antenna).reshape(-1),
                    prior_lo=_f64(spec.prior_lo), prior_hi=_f64(spec.prior_hi),
                    fixed_theta=_f64(spec.fixed_theta))
        rb0 = getattr(spec, "rb_theta0", None)
        rbe = getattr(spec, "rb_edges", None)
        keep["rb_theta0"] = None if rb0 is None else _f64(rb0)
        keep["rb_edges"] = None if rbe is None else np.ascontiguousarray(rbe, dtype=np.int32)
        self.keep = keep
        self.s = EventDesc(int(spec.n_bins), int(spec.n_det), int(spec.ndim), int(spec.like_kind),
                           float(spec.f_lo), float(spec.df), _ptr(keep["data"]),
                           _ptr(keep["psd"]), _ptr(keep["det_tensor"]), _ptr(keep["det_loc"]),
                           _ptr(keep["fixed_antenna"]), _ptr(keep["prior_lo"]),
                           _ptr(keep["prior_hi"]), _ptr(keep["fixed_theta"]), float(spec.gmst),
                           float(spec.toy_sigma), _ptr(keep["rb_theta0"]),
                           None if keep["rb_edges"] is None else
                           keep["rb_edges"].ctypes.data_as(C.POINTER(C.c_int32)),
                           0 if keep["rb_edges"] is None else len(keep["rb_edges"]) - 1, 0)


def _check(status: int, ctx=None, where=""):
    if status != NS_OK:
        msg = lib().ns_last_error(ctx).decode()
        raise NSError(status, f"{where}: {msg}" if where else msg)


def signal(spec, theta) -> np.ndarray:
    """Detector strain h_d(f_k) for theta, computed by the library's kernels;
    complex128 [n_det, n_bins]."""
    d = _Desc(spec)
    th = _f64(theta)
    out = np.zeros((spec.n_det, spec.n_bins, 2))
    _check(lib().ns_signal(C.byref(d.s), _ptr(th), _ptr(out)), None, "ns_signal")
    return out[..., 0] + 1j * out[..., 1]


def signal_noalloc(spec, theta) -> np.ndarray:
    """signal() through ns_signal_noalloc (no device allocation: a fixed
    per-GPU scratch array; at most 65536 bins)."""
    d = _Desc(spec)
    th = _f64(theta)
    out = np.zeros((spec.n_det, spec.n_bins, 2))
    _check(lib().ns_signal_noalloc(C.byref(d.s), _ptr(th), _ptr(out)), None, "ns_signal_noalloc")
    return out[..., 0] + 1j * out[..., 1]


def _stream_handle(stream) -> Optional[int]:
    if stream is None:
        return None
    if isinstance(stream, int):
        return stream
    return int(stream.cuda_stream)  # torch.cuda.Stream on ROCm is a hipStream_t


class Context:
    """One sampler context over one or more events (ns_init ... ns_free)."""

    def __init__(self, events: Sequence, datas: Sequence, *, n_live, num_delete, naccept, maxmcmc,
                 walk0=100, term_kind=0, term_thr=0.1, delay=-1.0, precision=NS_FP64, seed=0,
                 stream=None, timing=False, graph=False, inner="walk"):
        self._descs = [_Desc(s, d) for s, d in zip(events, datas)]
        arr = (EventDesc * len(self._descs))(*[d.s for d in self._descs])
        self.cfg = Config(int(n_live), int(num_delete), int(naccept), int(maxmcmc), int(walk0),
                          int(term_kind), float(delay), float(term_thr), int(precision),
                          (NS_FLAG_TIMING if timing else 0) | (NS_FLAG_GRAPH if graph else 0),
                          int(seed), _stream_handle(stream))
        h = C.c_void_p()
        st = lib().ns_init(C.byref(h), C.byref(self.cfg), arr, len(self._descs))
        _check(st, None, "ns_init")
        self.h = h
        if inner != "walk":
            self.set_inner(inner)
        self.n_live = int(n_live)
        self.ndim = int(events[0].ndim)
        self.n_events = len(self._descs)

    def close(self):
        if getattr(self, "h", None):
            lib().ns_free(self.h)
            self.h = None

    __del__ = close

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def _ck(self, st, where):
        _check(st, self.h, where)

    def step(self, k: int = 0, walk: int = 0):
        self._ck(lib().ns_step(self.h, int(k), int(walk)), "ns_step")

    def loglike_batch(self, event: int, theta, out, precision=NS_FP64):
        """theta: device tensor [n, 11] float64; out: device tensor [n] float64."""
        n = int(theta.shape[0])
        assert theta.is_contiguous() and out.is_contiguous() and out.numel() >= n
        self._ck(lib().ns_loglike_batch(self.h, int(event), C.c_void_p(theta.data_ptr()), n,
                                        C.c_void_p(out.data_ptr()), int(precision)),
                 "ns_loglike_batch")

    def loglike_batch_u(self, event: int, u, out, precision=NS_FP64):
        n = int(u.shape[0])
        assert u.is_contiguous() and out.is_contiguous() and out.numel() >= n
        self._ck(lib().ns_loglike_batch_u(self.h, int(event), C.c_void_p(u.data_ptr()), n,
                                          C.c_void_p(out.data_ptr()), int(precision)),
                 "ns_loglike_batch_u")

    def theta_from_u(self, event: int, u, theta):
        """u: device tensor [n, ndim] float64 -> theta: device tensor [n, 11] float64."""
        n = int(u.shape[0])
        assert u.is_contiguous() and theta.is_contiguous() and theta.numel() >= 11 * n
        self._ck(lib().ns_theta_from_u(self.h, int(event), C.c_void_p(u.data_ptr()), n,
                                       C.c_void_p(theta.data_ptr())), "ns_theta_from_u")

    def evidence(self, event: int = 0) -> dict:
        ev = Evidence()
        self._ck(lib().ns_evidence(self.h, int(event), C.byref(ev)), "ns_evidence")
        return ev.to_dict()

    def live(self, event: int = 0):
        u = np.zeros((self.n_live, self.ndim))
        L = np.zeros(self.n_live)
        self._ck(lib().ns_get_live(self.h, int(event), _ptr(u), _ptr(L)), "ns_get_live")
        return u, L

    def chain_stats(self, event: int = 0) -> np.ndarray:
        """Counts of each chain of the last batch: [k][4] int64 = accepts,
        exact calls, out-of-cube steps, discarded speculative evaluations."""
        out = np.zeros((self.n_live, 4), dtype=np.int64)
        n = C.c_int32()
        self._ck(lib().ns_get_chain_stats(self.h, int(event), out.ctypes.data_as(C.POINTER(C.c_int64)),
                                          self.n_live, C.byref(n)), "ns_get_chain_stats")
        return out[:n.value]

    def logz_replicates(self, event: int = 0, R: int = 200, seed: int = 0, uniforms=None):
        """log Z of R replicates with random prior-volume shrinkages
        (ns_logz_replicates); uniforms: optional device tensor [R][n_dead].
        Returns a float64 device tensor [R]."""
        import torch
        out = torch.empty(int(R), dtype=torch.float64, device="cuda")
        up = None if uniforms is None else C.c_void_p(uniforms.data_ptr())
        if uniforms is not None:
            assert uniforms.is_contiguous() and uniforms.dtype == torch.float64
        self._ck(lib().ns_logz_replicates(self.h, int(event), int(R), C.c_uint64(seed), up,
                                          C.c_void_p(out.data_ptr())), "ns_logz_replicates")
        return out

    def set_live(self, event: int, u, L):
        u = _f64(u).reshape(self.n_live, self.ndim)
        L = _f64(L).reshape(self.n_live)
        self._ck(lib().ns_set_live(self.h, int(event), _ptr(u), _ptr(L)), "ns_set_live")

    def dead(self, event: int = 0, max_rows: Optional[int] = None):
        if max_rows is None:
            max_rows = int(self.evidence(event)["n_dead"])
        u = np.zeros((max_rows, self.ndim)); L = np.zeros(max_rows)
        lw = np.zeros(max_rows); nl = np.zeros(max_rows)
        n = C.c_int64()
        self._ck(lib().ns_get_dead(self.h, int(event), int(max_rows), _ptr(u), _ptr(L), _ptr(lw),
                                   _ptr(nl), C.byref(n)), "ns_get_dead")
        r = n.value
        return u[:r], L[:r], lw[:r], nl[:r]

    def checkpoint(self) -> bytes:
        """The sampler state (live set, dead points, evidence accumulators,
        walk length, counters, batch index) as bytes for restore()."""
        n = C.c_int64()
        self._ck(lib().ns_checkpoint_size(self.h, C.byref(n)), "ns_checkpoint_size")
        buf = C.create_string_buffer(n.value)
        w = C.c_int64()
        self._ck(lib().ns_checkpoint(self.h, buf, n.value, C.byref(w)), "ns_checkpoint")
        return buf.raw[:w.value]

    def restore(self, data: bytes):
        """Load a checkpoint() of a context with the same events and sampler
        configuration; the run then continues exactly as the checkpointed one."""
        buf = C.create_string_buffer(bytes(data), len(data))
        self._ck(lib().ns_restore(self.h, buf, len(data)), "ns_restore")

    def autotune(self, cache_path: Optional[str] = None, trial_walk: int = 64) -> int:
        ch = C.c_int32()
        self._ck(lib().ns_autotune(self.h, cache_path.encode() if cache_path else None,
                                   int(trial_walk), C.byref(ch)), "ns_autotune")
        return ch.value

    def set_inner(self, inner: str):
        """Inner kernel of the chains: "walk" (acceptance walk) or "hrss"
        (hit-and-run slice sampling)."""
        kinds = {"walk": NS_INNER_WALK, "hrss": NS_INNER_HRSS}
        if inner not in kinds:
            raise ValueError(f"unknown inner kernel {inner!r}")
        self._ck(lib().ns_set_inner(self.h, kinds[inner]), "ns_set_inner")

    def set_waves_per_chain(self, wpc: int):
        self._ck(lib().ns_set_waves_per_chain(self.h, int(wpc)), "ns_set_waves_per_chain")

    def timing(self, reset: bool = False) -> dict:
        t = Timing()
        self._ck(lib().ns_timing(self.h, C.byref(t), 1 if reset else 0), "ns_timing")
        return {name: getattr(t, name) for name, _ in t._fields_}

    # ---- learned surrogate
    MLP_NPARAM = 134913

    def surrogate_init(self, seed: int = 0, max_rows: int = 4096):
        self._ck(lib().ns_surrogate_init(self.h, int(seed), int(max_rows)), "ns_surrogate_init")

    def surrogate_set_params(self, params):
        p = np.ascontiguousarray(np.asarray(params, dtype=np.float32))
        self._ck(lib().ns_surrogate_set_params(self.h, p.ctypes.data_as(C.POINTER(C.c_float)),
                                               p.size), "ns_surrogate_set_params")

    def surrogate_get_params(self) -> np.ndarray:
        p = np.zeros(self.MLP_NPARAM, dtype=np.float32)
        self._ck(lib().ns_surrogate_get_params(self.h, p.ctypes.data_as(C.POINTER(C.c_float)),
                                               p.size), "ns_surrogate_get_params")
        return p

    def surrogate_set_norm(self, mu: float, sigma: float, clip: float = -1e300,
                           top: float = math.inf):
        """Target map and normalisation: predictions are mu + sigma s(u) with
        top = inf, else top - exp(-(mu + sigma s(u))) (the log-gap map)."""
        self._ck(lib().ns_surrogate_set_norm(self.h, float(mu), float(sigma), float(clip),
                                             float(top)), "ns_surrogate_set_norm")

    def surrogate_get_norm(self):
        a, b, c, t = C.c_double(), C.c_double(), C.c_double(), C.c_double()
        self._ck(lib().ns_surrogate_get_norm(self.h, C.byref(a), C.byref(b), C.byref(c),
                                             C.byref(t)), "ns_surrogate_get_norm")
        return a.value, b.value, c.value, t.value

    def surrogate_set_input_norm(self, mean, stdev):
        m = _f64(mean); sd = _f64(stdev)
        assert m.size == self.ndim and sd.size == self.ndim
        self._ck(lib().ns_surrogate_set_input_norm(self.h, _ptr(m), _ptr(sd)),
                 "ns_surrogate_set_input_norm")

    def surrogate_get_input_norm(self):
        m = np.zeros(self.ndim); sd = np.zeros(self.ndim)
        self._ck(lib().ns_surrogate_get_input_norm(self.h, _ptr(m), _ptr(sd)),
                 "ns_surrogate_get_input_norm")
        return m, sd

    def surrogate_state(self):
        """Everything needed to load the trained network into another context."""
        return dict(params=self.surrogate_get_params(), norm=self.surrogate_get_norm(),
                    input_norm=self.surrogate_get_input_norm())

    def surrogate_load(self, state, seed=0, max_rows=64):
        self.surrogate_init(seed=seed, max_rows=max_rows)
        self.surrogate_set_params(state["params"])
        self.surrogate_set_norm(*state["norm"])
        self.surrogate_set_input_norm(*state["input_norm"])

    def surrogate_predict(self, u, out):
        n = int(u.shape[0])
        assert u.is_contiguous() and out.is_contiguous()
        self._ck(lib().ns_surrogate_predict(self.h, C.c_void_p(u.data_ptr()), n,
                                            C.c_void_p(out.data_ptr())), "ns_surrogate_predict")

    def surrogate_loss_grad(self, u, logl):
        n = int(u.shape[0])
        g = np.zeros(self.MLP_NPARAM, dtype=np.float32)
        loss = C.c_double()
        self._ck(lib().ns_surrogate_loss_grad(self.h, C.c_void_p(u.data_ptr()),
                                              C.c_void_p(logl.data_ptr()), n,
                                              g.ctypes.data_as(C.POINTER(C.c_float)),
                                              C.byref(loss)), "ns_surrogate_loss_grad")
        return loss.value, g

    def surrogate_train(self, u, logl, steps: int, batch: int = 4096, lr: float = 1e-3,
                        clip: float = -1e300, top: float = math.inf) -> float:
        """Fit the network to the pairs (u, logl); a finite top selects the
        log-gap target map (top must exceed every training target)."""
        loss = C.c_double()
        self._ck(lib().ns_surrogate_train(self.h, C.c_void_p(u.data_ptr()),
                                          C.c_void_p(logl.data_ptr()), int(u.shape[0]),
                                          int(steps), int(batch), float(lr), float(clip),
                                          float(top), C.byref(loss)), "ns_surrogate_train")
        return loss.value

    def surrogate_attach(self, margin: float = 5.0, temperature: float = 1.0, floor: float = 0.0):
        self._ck(lib().ns_surrogate_attach(self.h, float(margin), float(temperature), float(floor)),
                 "ns_surrogate_attach")

    def surrogate_detach(self):
        self._ck(lib().ns_surrogate_detach(self.h), "ns_surrogate_detach")

    def harvest(self, capacity: int):
        self._ck(lib().ns_harvest(self.h, int(capacity)), "ns_harvest")

    def harvest_copy(self, u_out, logl_out) -> int:
        n = C.c_int64()
        self._ck(lib().ns_harvest_copy(self.h, C.c_void_p(u_out.data_ptr()),
                                       C.c_void_p(logl_out.data_ptr()), int(logl_out.shape[0]),
                                       C.byref(n)), "ns_harvest_copy")
        return n.value

    def converged(self, event: int = 0) -> bool:
        return bool(self.evidence(event)["converged"])


def inject(spec):
    """Build event data d = h(theta) + n with the library's waveform, rescaling
    the distance so the optimal network SNR equals spec.target_snr (the SNR is
    read from the library's own likelihood: with d = h, log Lambda(theta) =
    rho^2 / 2).  Returns (data, theta_injected, fixed_theta)."""
    import dataclasses
    th = np.array(spec.theta_inj, dtype=np.float64)
    fixed = np.array(spec.fixed_theta, dtype=np.float64)
    if spec.like_kind not in (NS_LIKE_GW, NS_LIKE_GW_RB):
        return np.zeros((spec.n_det, spec.n_bins), np.complex128), th, fixed
    # the signal and its SNR come from the exact likelihood of the same event
    spec = dataclasses.replace(spec, like_kind=NS_LIKE_GW, rb_theta0=None, rb_edges=None)
    if spec.target_snr > 0:
        h = signal(spec, th)
        rho2 = 2.0 * _loglike_host(spec, h, th)
        th[4] = th[4] * np.sqrt(rho2) / spec.target_snr
    fixed[4] = th[4]
    spec2 = dataclasses.replace(spec, fixed_theta=fixed)
    data = signal(spec2, th) + np.asarray(spec.noise)
    return data, th, fixed


def _loglike_host(spec, data, theta) -> float:
    """log Lambda of one physical theta through the library (device round trip)."""
    import torch
    with Context([spec], [data], n_live=3, num_delete=1, naccept=1, maxmcmc=1, walk0=1) as ctx:
        t = torch.tensor(np.asarray(theta, np.float64)[None, :], device="cuda")
        o = torch.empty(1, dtype=torch.float64, device="cuda")
        ctx.loglike_batch(0, t, o)
        torch.cuda.synchronize()
        return float(o.cpu()[0])


def n_live_for_batch(n_sequential: int, frac: float = 0.5) -> int:
    """Live points for a batched run that match the per-deletion volume
    shrinkage of a sequential run (Sec. 3.2.1): k / n_seq = ln(n / (n - k))
    with k = frac * n, i.e. n = n_seq * (-ln(1 - frac)) / frac (2 ln 2 n_seq
    at frac = 1/2)."""
    return int(round(n_sequential * -np.log1p(-frac) / frac))
