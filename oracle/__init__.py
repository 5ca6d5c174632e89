"""CPU oracle for the acceptance-walk nested sampler (test infrastructure).

A plain FP64 implementation in C (``nsmi_oracle.c``) plus thin ctypes
marshalling and a few numpy helpers.  Only the tests, the smoke check and the
CPU-baseline leg of ``bench.py`` may import this package; the product path
(the HIP library and its binding) never does, and shares no code with it.

Functions without an independent pin are marked "parity unpinned" in their
docstring; every other function is pinned by a test under ``tests/`` against
closed forms, identities, numpy's Philox, brute force or quadrature.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "nsmi_oracle.c")
_SRCS = [_SRC, os.path.join(_HERE, "nsmi_mlp.c")]
_LIB_PATH = os.path.join(_HERE, "libnsmi_oracle.so")
_LIB = None

NPAR = 11
D = C.POINTER(C.c_double)


def build(verbose: bool = False) -> str:
    """Compile the oracle with gcc: -O2, IEEE semantics (no fast-math, no
    floating-point contraction), OpenMP across independent chains."""
    cmd = ["gcc", "-O2", "-std=gnu11", "-fno-fast-math", "-ffp-contract=off", "-fopenmp",
           "-fPIC", "-shared", *_SRCS, "-o", _LIB_PATH + ".tmp", "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.check_call(cmd)
    os.replace(_LIB_PATH + ".tmp", _LIB_PATH)
    return _LIB_PATH


def lib():
    global _LIB
    if _LIB is None:
        if not os.path.exists(_LIB_PATH) or any(
                os.path.getmtime(_LIB_PATH) < os.path.getmtime(f) for f in _SRCS):
            build()
        _LIB = C.CDLL(_LIB_PATH)
        _declare(_LIB)
    return _LIB


class _Event(C.Structure):
    _fields_ = [("n_bins", C.c_int32), ("n_det", C.c_int32), ("ndim", C.c_int32),
                ("like_kind", C.c_int32), ("f_lo", C.c_double), ("df", C.c_double),
                ("data", D), ("psd", D), ("det_tensor", D), ("det_loc", D),
                ("fixed_antenna", D), ("prior_lo", D), ("prior_hi", D), ("fixed_theta", D),
                ("gmst", C.c_double), ("toy_sigma", C.c_double),
                ("rb_theta0", D), ("rb_edges", C.POINTER(C.c_int32)), ("rb_bins", C.c_int32),
                ("rb_pad", C.c_int32)]


class _WalkStats(C.Structure):
    _fields_ = [("n_acc", C.c_int64), ("n_calls", C.c_int64), ("n_oob", C.c_int64)]


class _Screen(C.Structure):
    _fields_ = [("params", D), ("in_mean", C.c_double * NPAR), ("in_sd", C.c_double * NPAR),
                ("mu", C.c_double), ("sigma", C.c_double), ("top", C.c_double),
                ("const_s", C.c_double), ("margin", C.c_double), ("temp", C.c_double),
                ("floor", C.c_double)]


class _DAStats(C.Structure):
    _fields_ = [("n_acc", C.c_int64), ("n_calls", C.c_int64), ("n_oob", C.c_int64),
                ("n_saved", C.c_int64), ("min_gap_screen", C.c_double),
                ("min_gap_L", C.c_double)]


def _declare(L):
    E = C.POINTER(_Event)
    V = C.c_void_p
    L.or_prior_transform.argtypes = [E, D, D]
    L.or_pn_coeffs.argtypes = [C.c_double] * 6 + [D]
    L.or_phase.argtypes = [D, C.c_double]
    L.or_phase.restype = C.c_double
    L.or_amplitude.argtypes = [D]
    L.or_amplitude.restype = C.c_double
    L.or_antenna.argtypes = [D, C.c_double, C.c_double, C.c_double, C.c_double, D, D]
    L.or_time_delay.argtypes = [D, C.c_double, C.c_double, C.c_double]
    L.or_time_delay.restype = C.c_double
    L.or_waveform.argtypes = [E, D, D]
    L.or_loglike_theta.argtypes = [E, D]
    L.or_loglike_theta.restype = C.c_double
    L.or_loglike_rb.argtypes = [E, D]
    L.or_loglike_rb.restype = C.c_double
    L.or_loglike_u.argtypes = [E, D]
    L.or_loglike_u.restype = C.c_double
    L.or_loglike_batch_u.argtypes = [E, D, C.c_int64, D]
    L.or_loglike_batch_theta.argtypes = [E, D, C.c_int64, D]
    L.or_philox4x64.argtypes = [C.POINTER(C.c_uint64), C.POINTER(C.c_uint64),
                                C.POINTER(C.c_uint64)]
    L.or_u01.argtypes = [C.c_uint64]
    L.or_u01.restype = C.c_double
    L.or_is_periodic.argtypes = [C.c_int, C.c_int]
    L.or_is_periodic.restype = C.c_int
    L.or_walk.argtypes = [E, D, C.c_int32, C.c_double, D, D, C.c_int32, C.c_uint64, C.c_int32,
                          C.c_int32, C.c_int64, C.POINTER(_WalkStats)]
    L.or_hrss.argtypes = [E, D, C.c_int32, C.c_double, D, D, C.c_int32, C.c_uint64, C.c_int32,
                          C.c_int32, C.c_int64, C.POINTER(_WalkStats)]
    L.or_tune_walk.argtypes = [C.c_int32, C.c_int64, C.c_int32, C.c_double, C.c_int32,
                               C.c_int32]
    L.or_tune_walk.restype = C.c_int32
    L.or_ns_create.argtypes = [E, C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_int32,
                               C.c_double, C.c_uint64]
    L.or_ns_create.restype = V
    L.or_ns_free.argtypes = [V]
    L.or_ns_set_live.argtypes = [V, D, D]
    L.or_ns_step.argtypes = [V, C.c_int32, C.c_int32]
    L.or_ns_step.restype = C.c_int
    L.or_ns_set_inner.argtypes = [V, C.c_int32]
    L.or_ns_set_inner.restype = C.c_int
    L.or_ns_evidence.argtypes = [V, D]
    L.or_ns_n_dead.argtypes = [V]
    L.or_ns_n_dead.restype = C.c_int64
    L.or_ns_W.argtypes = [V]
    L.or_ns_W.restype = C.c_int32
    L.or_ns_set_W.argtypes = [V, C.c_int32]
    L.or_ns_batch.argtypes = [V]
    L.or_ns_batch.restype = C.c_int64
    L.or_ns_get_live.argtypes = [V, D, D]
    L.or_ns_get_dead.argtypes = [V, D, D, D, D]
    L.or_ns_stats.argtypes = [V, C.POINTER(C.c_int64)]
    L.or_ns_last_Lstar.argtypes = [V]
    L.or_ns_last_Lstar.restype = C.c_double
    L.or_num_threads.restype = C.c_int
    L.or_de_gamma.argtypes = [C.c_double, D, C.c_int]
    L.or_de_gamma.restype = C.c_double
    L.or_mlp_num_params.restype = C.c_int64
    L.or_mlp_forward.argtypes = [D, D, C.c_int64, D]
    L.or_mlp_loss_grad.argtypes = [D, D, D, C.c_int64, D]
    L.or_mlp_loss_grad.restype = C.c_double
    L.or_adam_step.argtypes = [D, D, D, D, C.c_int64, C.c_int64, C.c_double, C.c_double,
                               C.c_double, C.c_double]
    S = C.POINTER(_Screen)
    L.or_mlp_eval1.argtypes = [D, D]
    L.or_mlp_eval1.restype = C.c_double
    L.or_screen_predict.argtypes = [S, C.c_int, D]
    L.or_screen_predict.restype = C.c_double
    L.or_screen_density.argtypes = [S, C.c_double, C.c_double]
    L.or_screen_density.restype = C.c_double
    L.or_walk_da.argtypes = [E, S, D, C.c_int32, C.c_double, D, D, C.c_int32, C.c_uint64,
                             C.c_int32, C.c_int32, C.c_int64, C.POINTER(_DAStats)]
    L.or_ns_set_screen.argtypes = [V, S]
    L.or_ns_n_saved.argtypes = [V]
    L.or_ns_n_saved.restype = C.c_int64
    L.or_ns_last_gaps.argtypes = [V, D, D, C.c_int32]
    L.or_ns_last_gaps.restype = C.c_int32
    L.or_ns_last_chains.argtypes = [V, C.POINTER(C.c_int64), C.c_int32]
    L.or_ns_last_chains.restype = C.c_int32


def _p(a: Optional[np.ndarray]):
    if a is None:
        return C.cast(None, D)
    return a.ctypes.data_as(D)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


class Event:
    """An event as the oracle sees it: grid, data, PSD, detectors, priors."""

    def __init__(self, *, f_lo, df, n_bins, n_det, ndim, data, psd, det_tensor=None,
                 det_loc=None, fixed_antenna=None, prior_lo, prior_hi, fixed_theta, gmst=0.0,
                 like_kind=0, toy_sigma=0.1, rb_theta0=None, rb_edges=None):
        data = np.asarray(data)
        if np.iscomplexobj(data):
            data = np.stack([data.real, data.imag], axis=-1)
        self._keep = dict(
            data=_f64(data).reshape(-1), psd=_f64(psd).reshape(-1),
            det_tensor=None if det_tensor is None else _f64(det_tensor).reshape(-1),
            det_loc=None if det_loc is None else _f64(det_loc).reshape(-1),
            fixed_antenna=None if fixed_antenna is None else _f64(fixed_antenna).reshape(-1),
            prior_lo=_f64(prior_lo), prior_hi=_f64(prior_hi), fixed_theta=_f64(fixed_theta),
            rb_theta0=None if rb_theta0 is None else _f64(rb_theta0),
            rb_edges=None if rb_edges is None else np.ascontiguousarray(rb_edges, dtype=np.int32))
        k = self._keep
        if like_kind == 2:
            e = k["rb_edges"]
            if (k["rb_theta0"] is None or e is None or len(e) < 2 or e[0] != 0
                    or e[-1] != int(n_bins) or np.any(np.diff(e) <= 0)):
                raise ValueError("relative binning needs rb_theta0 and increasing rb_edges "
                                 "from 0 to n_bins")
        self.n_bins, self.n_det, self.ndim = int(n_bins), int(n_det), int(ndim)
        self.f_lo, self.df = float(f_lo), float(df)
        self.s = _Event(self.n_bins, self.n_det, self.ndim, int(like_kind), self.f_lo, self.df,
                        _p(k["data"]), _p(k["psd"]), _p(k["det_tensor"]), _p(k["det_loc"]),
                        _p(k["fixed_antenna"]), _p(k["prior_lo"]), _p(k["prior_hi"]),
                        _p(k["fixed_theta"]), float(gmst), float(toy_sigma),
                        _p(k["rb_theta0"]),
                        None if k["rb_edges"] is None else
                        k["rb_edges"].ctypes.data_as(C.POINTER(C.c_int32)),
                        0 if k["rb_edges"] is None else len(k["rb_edges"]) - 1, 0)
        self.like_kind = int(like_kind)

    @property
    def ref(self):
        return C.byref(self.s)

    def with_data(self, data) -> "Event":
        k = self._keep
        return Event(f_lo=self.f_lo, df=self.df, n_bins=self.n_bins, n_det=self.n_det,
                     ndim=self.ndim, data=data, psd=k["psd"].reshape(self.n_det, self.n_bins),
                     det_tensor=k["det_tensor"], det_loc=k["det_loc"],
                     fixed_antenna=k["fixed_antenna"], prior_lo=k["prior_lo"],
                     prior_hi=k["prior_hi"], fixed_theta=k["fixed_theta"], gmst=self.s.gmst,
                     like_kind=self.s.like_kind, toy_sigma=self.s.toy_sigma,
                     rb_theta0=k["rb_theta0"], rb_edges=k["rb_edges"])


# ---------------------------------------------------------------- elementary pieces

def prior_transform(ev: Event, u) -> np.ndarray:
    u = _f64(u)
    th = np.zeros(NPAR)
    lib().or_prior_transform(ev.ref, _p(u), _p(th))
    return th


def pn_coeffs(eta, x, chis, chia, Ms, f) -> np.ndarray:
    out = np.zeros(8)
    lib().or_pn_coeffs(eta, x, chis, chia, Ms, f, _p(out))
    return out


def phase(theta, f) -> float:
    return lib().or_phase(_p(_f64(theta)), float(f))


def amplitude(theta) -> float:
    return lib().or_amplitude(_p(_f64(theta)))


def antenna(tensor, ra, dec, psi, gmst=0.0):
    fp, fx = C.c_double(), C.c_double()
    lib().or_antenna(_p(_f64(tensor)), ra, dec, psi, gmst, C.byref(fp), C.byref(fx))
    return fp.value, fx.value


def time_delay(loc, ra, dec, gmst=0.0) -> float:
    return lib().or_time_delay(_p(_f64(loc)), ra, dec, gmst)


def waveform(ev: Event, theta) -> np.ndarray:
    """Detector strain h_d(f_k) as complex128 [n_det, n_bins]."""
    out = np.zeros((ev.n_det, ev.n_bins, 2))
    lib().or_waveform(ev.ref, _p(_f64(theta)), _p(out))
    return out[..., 0] + 1j * out[..., 1]


def loglike_theta(ev: Event, theta) -> float:
    """Exact Whittle log-likelihood ratio (whatever the event's kind)."""
    return lib().or_loglike_theta(ev.ref, _p(_f64(theta)))


def loglike_rb(ev: Event, theta) -> float:
    """Relative-binning log-likelihood ratio (the event must carry rb_theta0
    and rb_edges)."""
    if ev.s.rb_bins < 1:
        raise ValueError("event has no relative-binning nodes")
    return lib().or_loglike_rb(ev.ref, _p(_f64(theta)))


def loglike_u(ev: Event, u) -> float:
    return lib().or_loglike_u(ev.ref, _p(_f64(u)))


def loglike_batch_theta(ev: Event, theta) -> np.ndarray:
    th = _f64(theta).reshape(-1, NPAR)
    out = np.zeros(th.shape[0])
    lib().or_loglike_batch_theta(ev.ref, _p(th), th.shape[0], _p(out))
    return out


def loglike_batch_u(ev: Event, u) -> np.ndarray:
    uu = _f64(u).reshape(-1, ev.ndim)
    out = np.zeros(uu.shape[0])
    lib().or_loglike_batch_u(ev.ref, _p(uu), uu.shape[0], _p(out))
    return out


def philox4x64(counter, key) -> np.ndarray:
    c = np.ascontiguousarray(np.asarray(counter, dtype=np.uint64))
    k = np.ascontiguousarray(np.asarray(key, dtype=np.uint64))
    out = np.zeros(4, dtype=np.uint64)
    P = C.POINTER(C.c_uint64)
    lib().or_philox4x64(c.ctypes.data_as(P), k.ctypes.data_as(P), out.ctypes.data_as(P))
    return out


def u01(r: int) -> float:
    return lib().or_u01(C.c_uint64(int(r)))


def walk(ev: Event, snapshot, Lstar, u0, L0, W, seed, event, slot, batch):
    """One acceptance-walk chain; returns (u, L, n_acc, n_calls, n_oob)."""
    S = _f64(snapshot).reshape(-1, ev.ndim)
    u = _f64(u0).copy()
    L = C.c_double(L0)
    st = _WalkStats()
    lib().or_walk(ev.ref, _p(S), S.shape[0], float(Lstar), _p(u), C.byref(L), int(W),
                  C.c_uint64(seed), int(event), int(slot), int(batch), C.byref(st))
    return u, L.value, st.n_acc, st.n_calls, st.n_oob


def hrss(ev: Event, snapshot, Lstar, u0, L0, W, seed, event, slot, batch):
    """One hit-and-run slice-sampling chain of W slice steps; returns
    (u, L, n_moves, n_calls, n_oob)."""
    S = _f64(snapshot).reshape(-1, ev.ndim)
    u = _f64(u0).copy()
    L = C.c_double(L0)
    st = _WalkStats()
    lib().or_hrss(ev.ref, _p(S), S.shape[0], float(Lstar), _p(u), C.byref(L), int(W),
                  C.c_uint64(seed), int(event), int(slot), int(batch), C.byref(st))
    return u, L.value, st.n_acc, st.n_calls, st.n_oob


class Screen:
    """Screen of the delayed-acceptance walk: the surrogate prediction
    s(u) = z^-1(mu + sigma MLP((u - in_mean) / in_sd)) (z^-1 the identity, or
    top - exp(-w) for a finite top), or a constant when params is None, and
    the density pi = floor + (1 - floor) sigmoid((s - L* + margin) / temp)."""

    def __init__(self, params=None, *, in_mean=None, in_sd=None, mu=0.0, sigma=1.0,
                 top=np.inf, const_s=0.0, margin=0.0, temp=1.0, floor=0.0):
        self._p = None if params is None else _f64(params).copy()
        if self._p is not None and self._p.size != mlp_num_params():
            raise ValueError("screen parameters have the wrong size")
        m = np.zeros(NPAR) if in_mean is None else np.resize(_f64(in_mean), NPAR)
        sd = np.ones(NPAR) if in_sd is None else np.resize(_f64(in_sd), NPAR)
        self.s = _Screen(_p(self._p), (C.c_double * NPAR)(*m), (C.c_double * NPAR)(*sd),
                         float(mu), float(sigma), float(top), float(const_s), float(margin),
                         float(temp), float(floor))

    @property
    def ref(self):
        return C.byref(self.s)

    def predict(self, ndim, u) -> np.ndarray:
        uu = _f64(u).reshape(-1, ndim)
        return np.array([lib().or_screen_predict(self.ref, ndim, _p(np.ascontiguousarray(r)))
                         for r in uu])

    def density(self, s_hat, Lstar) -> float:
        return lib().or_screen_density(self.ref, float(s_hat), float(Lstar))


def walk_da(ev: Event, screen: Screen, snapshot, Lstar, u0, L0, W, seed, event, slot, batch):
    """One delayed-acceptance chain; returns (u, L, stats) with stats the
    counts (n_acc, n_calls, n_oob, n_saved) and the smallest decision gaps
    (min_gap_screen, min_gap_L)."""
    S = _f64(snapshot).reshape(-1, ev.ndim)
    u = _f64(u0).copy()
    L = C.c_double(L0)
    st = _DAStats()
    lib().or_walk_da(ev.ref, screen.ref, _p(S), S.shape[0], float(Lstar), _p(u), C.byref(L),
                     int(W), C.c_uint64(seed), int(event), int(slot), int(batch), C.byref(st))
    stats = dict(n_acc=st.n_acc, n_calls=st.n_calls, n_oob=st.n_oob, n_saved=st.n_saved,
                 min_gap_screen=st.min_gap_screen, min_gap_L=st.min_gap_L)
    return u, L.value, stats


def de_gamma(u_mode, ug, ndim) -> float:
    """Differential-evolution scale for one step from its uniforms."""
    return lib().or_de_gamma(float(u_mode), _p(_f64(ug)), int(ndim))


def tune_walk(W, sum_acc, k, delay, naccept, maxmcmc) -> int:
    return lib().or_tune_walk(W, sum_acc, k, delay, naccept, maxmcmc)


def num_threads() -> int:
    return lib().or_num_threads()


# ---------------------------------------------------------------- sampler

class NS:
    """Batched nested sampling run (oracle); inner kernel "walk" (acceptance
    walk) or "hrss" (hit-and-run slice sampling)."""

    def __init__(self, ev: Event, *, n_live, naccept, maxmcmc, walk0=100, delay=None, seed=0,
                 event_id=0, inner="walk"):
        self.ev = ev
        self.n_live = int(n_live)
        self.ndim = ev.ndim
        if delay is None:
            delay = max(n_live / 10.0 - 1.0, 0.0)
        self.h = lib().or_ns_create(ev.ref, int(event_id), self.n_live, int(naccept),
                                    int(maxmcmc), int(walk0), float(delay), C.c_uint64(seed))
        if inner not in ("walk", "hrss"):
            raise ValueError(f"unknown inner kernel {inner!r}")
        lib().or_ns_set_inner(self.h, 1 if inner == "hrss" else 0)

    def __del__(self):
        if getattr(self, "h", None):
            lib().or_ns_free(self.h)
            self.h = None

    def set_screen(self, screen: Optional["Screen"]):
        """Delayed acceptance through `screen` in later walks (None: plain)."""
        self._screen = screen  # kept alive while the sampler uses it
        lib().or_ns_set_screen(self.h, None if screen is None else screen.ref)

    @property
    def n_saved(self) -> int:
        return int(lib().or_ns_n_saved(self.h))

    def last_gaps(self):
        """Smallest decision gaps (screen, exact) of each chain of the last
        batch with a screen (inf without one)."""
        gs = np.zeros(self.n_live)
        gl = np.zeros(self.n_live)
        n = lib().or_ns_last_gaps(self.h, _p(gs), _p(gl), self.n_live)
        return gs[:n], gl[:n]

    def last_chains(self) -> np.ndarray:
        """Counts of each chain of the last batch: [k][3] accepts, calls,
        out-of-cube steps."""
        out = np.zeros((self.n_live, 3), dtype=np.int64)
        n = lib().or_ns_last_chains(self.h, out.ctypes.data_as(C.POINTER(C.c_int64)), self.n_live)
        return out[:n]

    def step(self, k, walk=0):
        rc = lib().or_ns_step(self.h, int(k), int(walk))
        if rc != 0:
            raise ValueError(f"oracle ns_step rejected k={k} (rc={rc})")

    def set_live(self, u, L):
        u = _f64(u).reshape(self.n_live, self.ndim)
        L = _f64(L).reshape(self.n_live)
        lib().or_ns_set_live(self.h, _p(u), _p(L))

    def live(self):
        u = np.zeros((self.n_live, self.ndim))
        L = np.zeros(self.n_live)
        lib().or_ns_get_live(self.h, _p(u), _p(L))
        return u, L

    def dead(self):
        n = lib().or_ns_n_dead(self.h)
        u = np.zeros((n, self.ndim)); L = np.zeros(n); lw = np.zeros(n); nl = np.zeros(n)
        lib().or_ns_get_dead(self.h, _p(u), _p(L), _p(lw), _p(nl))
        return u, L, lw, nl

    def evidence(self) -> dict:
        out = np.zeros(7)
        lib().or_ns_evidence(self.h, _p(out))
        return dict(logZ_dead=out[0], logZ=out[1], dlogZ=out[2], log_frac=out[3], H=out[4],
                    logX=out[5], logZ_err=out[6])

    @property
    def W(self) -> int:
        return lib().or_ns_W(self.h)

    @W.setter
    def W(self, w):
        lib().or_ns_set_W(self.h, int(w))

    @property
    def batch(self) -> int:
        return lib().or_ns_batch(self.h)

    def stats(self) -> dict:
        out = np.zeros(10, dtype=np.int64)
        lib().or_ns_stats(self.h, out.ctypes.data_as(C.POINTER(C.c_int64)))
        keys = ("calls", "accepts", "oob", "steps", "last_acc", "last_calls", "last_oob",
                "last_W", "last_k", "capped")
        return dict(zip(keys, (int(x) for x in out)))

    @property
    def last_Lstar(self) -> float:
        return lib().or_ns_last_Lstar(self.h)

    def converged(self, term_kind: int, thr: float) -> bool:
        e = self.evidence()
        if term_kind == 0:
            return e["dlogZ"] < thr
        return e["log_frac"] < np.log(thr)

    def run(self, k, term_kind, thr, max_batches=100000):
        for _ in range(max_batches):
            if self.converged(term_kind, thr):
                break
            self.step(k)
        return self.evidence()


def logz_spread(dead_L, dead_nlive, live_L, R=200, seed=0, uniforms=None, return_all=False):
    """Spread of logZ from the statistical uncertainty of the dead-point
    volumes (Sec. 5 / App. A): each replicate replaces every expected
    shrinkage -1/n_i by log(t_i), t_i ~ Beta(n_i, 1), i.e. log(U)/n_i, and
    re-accumulates the evidence including the final live points.
    uniforms: optional [R][n_dead] array of the U (drawn from numpy's
    generator otherwise).  Returns (mean, std) over R replicates, or with
    return_all the R values."""
    rng = np.random.default_rng(seed)
    dead_L = np.asarray(dead_L); nl = np.asarray(dead_nlive)
    n_live = len(live_L)
    lmx = np.max(live_L)
    lme = lmx + np.log(np.mean(np.exp(np.asarray(live_L) - lmx)))
    out = np.empty(R)
    for r in range(R):
        u = rng.random(len(nl)) if uniforms is None else np.asarray(uniforms[r], dtype=np.float64)
        dlx = np.log(u) / nl
        logX = np.concatenate([[0.0], np.cumsum(dlx)])
        logw = logX[:-1] + np.log(-np.expm1(dlx))
        t = dead_L + logw
        m = max(t.max(), logX[-1] + lme)
        out[r] = m + np.log(np.sum(np.exp(t - m)) + np.exp(logX[-1] + lme - m))
    del n_live
    if return_all:
        return out
    return float(out.mean()), float(out.std(ddof=1))


def make_data(ev_nodata: Event, theta_signal, noise) -> np.ndarray:
    """Event data d = h(theta) + n, the signal from the oracle's own waveform."""
    return waveform(ev_nodata, theta_signal) + np.asarray(noise)


def event_from_spec(spec, data=None) -> Event:
    """Build an oracle Event from an ``inputs.EventSpec`` (data defaults to
    zeros; use ``build_event`` to inject the signal)."""
    if data is None:
        data = np.zeros((spec.n_det, spec.n_bins), np.complex128)
    return Event(f_lo=spec.f_lo, df=spec.df, n_bins=spec.n_bins, n_det=spec.n_det,
                 ndim=spec.ndim, data=data, psd=spec.psd, det_tensor=spec.det_tensor,
                 det_loc=spec.det_loc, fixed_antenna=spec.fixed_antenna,
                 prior_lo=spec.prior_lo, prior_hi=spec.prior_hi, fixed_theta=spec.fixed_theta,
                 gmst=spec.gmst, like_kind=spec.like_kind, toy_sigma=spec.toy_sigma,
                 rb_theta0=getattr(spec, "rb_theta0", None), rb_edges=getattr(spec, "rb_edges", None))


def optimal_snr2(ev: Event, theta) -> float:
    """sum_d <h_d|h_d> by direct summation over bins."""
    h = waveform(ev, theta)
    psd = ev._keep["psd"].reshape(ev.n_det, ev.n_bins)
    return float(4.0 * ev.df * np.sum(np.abs(h) ** 2 / psd))


def build_event(spec):
    """Inject the signal with the oracle's waveform: rescale dL so the optimal
    network SNR equals spec.target_snr, then d = h + n.  Returns
    (event, theta_injected, data)."""
    base = event_from_spec(spec)
    th = np.array(spec.theta_inj, dtype=np.float64)
    if spec.like_kind == 0 and spec.target_snr > 0:
        rho = np.sqrt(optimal_snr2(base, th))
        th[4] = th[4] * rho / spec.target_snr
    fixed = np.array(spec.fixed_theta, dtype=np.float64)
    fixed[4] = th[4]
    spec2 = _replace_fixed(spec, fixed)
    base2 = event_from_spec(spec2)
    if spec.like_kind == 0:
        data = make_data(base2, th, spec.noise)
    else:
        data = np.zeros((spec.n_det, spec.n_bins), np.complex128)
    return event_from_spec(spec2, data), th, data


def _replace_fixed(spec, fixed):
    import dataclasses
    return dataclasses.replace(spec, fixed_theta=fixed)


# ---------------------------------------------------------------- surrogate MLP

MLP_IN, MLP_H = 11, 256


def mlp_num_params() -> int:
    return int(lib().or_mlp_num_params())


def mlp_forward(params, x) -> np.ndarray:
    """Network output for x [n, 11] (inputs beyond the sampled dimension are 0)."""
    p = _f64(params)
    xx = _f64(x).reshape(-1, MLP_IN)
    y = np.zeros(xx.shape[0])
    lib().or_mlp_forward(_p(p), _p(xx), xx.shape[0], _p(y))
    return y


def mlp_loss_grad(params, x, t):
    """Mean squared error and its gradient (same layout as params)."""
    p = _f64(params)
    xx = _f64(x).reshape(-1, MLP_IN)
    tt = _f64(t).reshape(-1)
    g = np.zeros_like(p)
    loss = lib().or_mlp_loss_grad(_p(p), _p(xx), _p(tt), xx.shape[0], _p(g))
    return loss, g


def adam_step(params, grad, m, v, t, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8):
    """In-place Adam update of params, m, v (float64 arrays)."""
    for a in (params, m, v):
        assert a.dtype == np.float64 and a.flags.c_contiguous
    g = _f64(grad)
    lib().or_adam_step(_p(params), _p(g), _p(m), _p(v), params.size, int(t), lr, beta1, beta2, eps)


def mlp_unpack(params):
    """Views W1 [256, 11], b1, W2 [256, 256], b2, W3, b3, W4 [1, 256], b4."""
    p = np.asarray(params)
    H, I = MLP_H, MLP_IN
    o = np.cumsum([0, H * I, H, H * H, H, H * H, H, H, 1])
    return (p[o[0]:o[1]].reshape(H, I), p[o[1]:o[2]], p[o[2]:o[3]].reshape(H, H), p[o[3]:o[4]],
            p[o[4]:o[5]].reshape(H, H), p[o[5]:o[6]], p[o[6]:o[7]].reshape(1, H), p[o[7]:o[8]])
