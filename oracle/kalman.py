"""ORACLE -- test infrastructure only.

ctypes wrapper around ``kalman.c`` (sequential augmented Kalman filter, RTS
smoother and prediction at arbitrary times, in long double), plus the
finite-difference gradient of its log-likelihood.  See ``kalman.c`` for the
sections of the paper each step follows.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "kalman.c")
_LIB_PATH = os.path.join(_HERE, "libgp_oracle.so")
_lib = None
_lock = threading.Lock()

_dp = ctypes.POINTER(ctypes.c_double)
_ip = ctypes.POINTER(ctypes.c_int32)


def build(force: bool = False) -> str:
    """Compile ``kalman.c`` into ``libgp_oracle.so`` next to it."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def lib():
    global _lib
    with _lock:
        if _lib is None:
            build()
            L = ctypes.CDLL(_LIB_PATH)
            L.oracle_term_discretise.argtypes = [ctypes.c_double] * 4 + [_dp, _dp]
            L.oracle_term_discretise.restype = ctypes.c_int
            L.oracle_greedy_slots.argtypes = [ctypes.c_int64, _dp, _dp, _ip, _ip]
            L.oracle_greedy_slots.restype = ctypes.c_int
            L.oracle_loglik.argtypes = [ctypes.c_int64, _dp, _dp, _dp, _dp, _ip, ctypes.c_int32, _dp, _dp, _dp, _ip,
                                        _dp, _dp, ctypes.c_double, ctypes.c_int32, _dp]
            L.oracle_loglik.restype = ctypes.c_int
            L.oracle_loglik_sqrt.argtypes = [ctypes.c_int64, _dp, _dp, _dp, _dp, _ip, ctypes.c_int32, _dp, _dp, _dp,
                                             _ip, _dp, _dp, ctypes.c_double, _dp]
            L.oracle_loglik_sqrt.restype = ctypes.c_int
            L.oracle_smooth.argtypes = [ctypes.c_int64, _dp, _dp, _dp, _dp, _ip, ctypes.c_int32, _dp, _dp, _dp, _ip,
                                        _dp, _dp, ctypes.c_double, ctypes.c_int64, _dp, _dp, _dp, _dp, _dp, _dp, _dp, _dp]
            L.oracle_smooth.restype = ctypes.c_int
            _lib = L
    return _lib


def _d(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(_dp)


class OracleError(RuntimeError):
    def __init__(self, code):
        super().__init__("oracle returned error code %d" % code)
        self.code = code


def term_discretise(omega0, quality, sigma, dt):
    """Augmented single-term transition (3x3) and process noise (3x3) over
    ``dt`` for state (x, xdot, z), unscaled coordinates."""
    phi = np.zeros(9)
    q = np.zeros(9)
    rc = lib().oracle_term_discretise(float(omega0), float(quality), float(sigma), float(dt), _d(phi)[1], _d(q)[1])
    if rc:
        raise OracleError(rc)
    return phi.reshape(3, 3), q.reshape(3, 3)


def greedy_slots(ts, te):
    ts, pts = _d(ts)
    te, pte = _d(te)
    slot = np.zeros(len(ts), dtype=np.int32)
    nj = np.zeros(1, dtype=np.int32)
    rc = lib().oracle_greedy_slots(len(ts), pts, pte, slot.ctypes.data_as(_ip), nj.ctypes.data_as(_ip))
    if rc:
        raise OracleError(rc)
    return slot, int(nj[0])


KINDS = {"sho": 0, "real": 1}


def _kinds(kinds, M):
    """Term kinds as an int32 array (0: SHO, 1: real exponential term), or
    (None, None) for all SHO."""
    if kinds is None:
        return None, None
    k = np.ascontiguousarray([KINDS.get(v, v) for v in kinds], dtype=np.int32)
    assert len(k) == M
    return k, k.ctypes.data_as(_ip)


def expand_instruments(instrument, amp=None, off=None):
    """Per-measurement amplitude and offset from per-instrument values:
    measurement n takes amp[instrument[n]] and off[instrument[n]] (Sec. 2.2,
    the observation matrix scaled per instrument; Sec. 3.2.3, labels)."""
    instrument = np.asarray(instrument, dtype=np.int64)
    a = None if amp is None else np.asarray(amp, dtype=np.float64)[instrument]
    c = None if off is None else np.asarray(off, dtype=np.float64)[instrument]
    return a, c


def _opt(a, n):
    if a is None:
        return None, None
    a = np.ascontiguousarray(a, dtype=np.float64)
    assert a.shape == (n,)
    return a, a.ctypes.data_as(_dp)


def _prep(ts, te, y, yerr, sigma, omega0, quality, slots):
    arrs = [_d(a) for a in (ts, te, y, yerr)]
    terms = [_d(np.atleast_1d(a)) for a in (sigma, omega0, quality)]
    sl = None
    slp = None
    if slots is not None:
        sl = np.ascontiguousarray(slots, dtype=np.int32)
        slp = sl.ctypes.data_as(_ip)
    return arrs, terms, sl, slp


def loglik_hilo(ts, te, y, yerr, sigma, omega0, quality, jitter=0.0, slots=None, extra_slots=0, kinds=None, amp=None,
                off=None):
    """Log-likelihood as a (hi, lo) double-double pair.  kinds: per term
    'sho' (default) or 'real' (sigma^2 exp(-omega0 |tau|), quality unused).
    amp, off: per-measurement amplitude a_n and offset c_n of the
    observation, y_n = a_n * (exposure average) + c_n + noise (default 1, 0)."""
    arrs, terms, sl, slp = _prep(ts, te, y, yerr, sigma, omega0, quality, slots)
    out = np.zeros(2)
    M = len(terms[0][0])
    n = len(arrs[0][0])
    kd, kp = _kinds(kinds, M)
    ad, ap = _opt(amp, n)
    od, op = _opt(off, n)
    rc = lib().oracle_loglik(n, arrs[0][1], arrs[1][1], arrs[2][1], arrs[3][1], slp, M, terms[0][1],
                             terms[1][1], terms[2][1], kp, ap, op, float(jitter), int(extra_slots), _d(out)[1])
    if rc:
        raise OracleError(rc)
    return float(out[0]), float(out[1])


def loglik_sqrt(ts, te, y, yerr, sigma, omega0, quality, jitter=0.0, slots=None, kinds=None, amp=None, off=None):
    """Log-likelihood by the square-root (Cholesky-factor) form of the same
    filter (QR time update, Givens array measurement update), long double."""
    arrs, terms, sl, slp = _prep(ts, te, y, yerr, sigma, omega0, quality, slots)
    out = np.zeros(2)
    M = len(terms[0][0])
    n = len(arrs[0][0])
    kd, kp = _kinds(kinds, M)
    ad, ap = _opt(amp, n)
    od, op = _opt(off, n)
    rc = lib().oracle_loglik_sqrt(n, arrs[0][1], arrs[1][1], arrs[2][1], arrs[3][1], slp, M, terms[0][1],
                                  terms[1][1], terms[2][1], kp, ap, op, float(jitter), _d(out)[1])
    if rc:
        raise OracleError(rc)
    return float(out[0]) + float(out[1])


def loglik(ts, te, y, yerr, sigma, omega0, quality, jitter=0.0, slots=None, extra_slots=0, kinds=None, amp=None,
           off=None):
    hi, lo = loglik_hilo(ts, te, y, yerr, sigma, omega0, quality, jitter, slots, extra_slots, kinds, amp, off)
    return hi + lo


def smooth(ts, te, y, yerr, sigma, omega0, quality, jitter=0.0, t_test=None, slots=None, terms=False, kinds=None,
           amp=None, off=None):
    """Returns (loglik, mean_test, var_test, mean_data, var_data), and with
    terms=True also the per-term latent posterior at t_test (term_mean,
    term_var, each [n_test, M]: H^m applied to the smoothed state, Appendix
    C, component-wise predictive means and variances).  mean_test/var_test
    are the latent process; mean_data/var_data the noise-free measured
    quantity a_n * (exposure average) + c_n."""
    want_terms = terms
    arrs, terms, sl, slp = _prep(ts, te, y, yerr, sigma, omega0, quality, slots)
    n = len(arrs[0][0])
    tt = np.zeros(0) if t_test is None else np.ascontiguousarray(t_test, dtype=np.float64)
    mt = np.zeros(len(tt))
    vt = np.zeros(len(tt))
    md = np.zeros(n)
    vd = np.zeros(n)
    out = np.zeros(2)
    M = len(terms[0][0])
    tm = np.zeros((len(tt), M))
    tv = np.zeros((len(tt), M))
    kd, kp = _kinds(kinds, M)
    ad, ap = _opt(amp, n)
    od, op = _opt(off, n)
    rc = lib().oracle_smooth(n, arrs[0][1], arrs[1][1], arrs[2][1], arrs[3][1], slp, M, terms[0][1], terms[1][1],
                             terms[2][1], kp, ap, op, float(jitter), len(tt), _d(tt)[1], _d(mt)[1], _d(vt)[1], _d(md)[1], _d(vd)[1],
                             _d(tm)[1] if want_terms else None, _d(tv)[1] if want_terms else None, _d(out)[1])
    if rc:
        raise OracleError(rc)
    if want_terms:
        return out[0] + out[1], mt, vt, md, vd, tm, tv
    return out[0] + out[1], mt, vt, md, vd


def loglik_grad_fd(ts, te, y, yerr, sigma, omega0, quality, jitter=0.0, rel_step=1e-6, slots=None, kinds=None, amp=None,
                   off=None):
    """Central finite differences of the log-likelihood with relative steps
    h_i = rel_step * |theta_i| in the natural parameters.  Returns the
    gradient ordered (d sigma_1..M, d omega0_1..M, d Q_1..M, d jitter).
    A zero jitter uses an absolute step of ``rel_step``."""
    sigma = np.atleast_1d(np.asarray(sigma, dtype=np.float64))
    omega0 = np.atleast_1d(np.asarray(omega0, dtype=np.float64))
    quality = np.atleast_1d(np.asarray(quality, dtype=np.float64))
    M = len(sigma)
    theta = np.concatenate([sigma, omega0, quality, [float(jitter)]])
    g = np.zeros_like(theta)

    def L(th):
        hi, lo = loglik_hilo(ts, te, y, yerr, th[:M], th[M:2 * M], th[2 * M:3 * M], th[3 * M], slots, kinds=kinds,
                             amp=amp, off=off)
        return hi, lo

    for i in range(len(theta)):
        h = rel_step * abs(theta[i]) if theta[i] != 0 else rel_step
        tp = theta.copy()
        tm = theta.copy()
        tp[i] += h
        tm[i] -= h
        if i == 3 * M and tm[i] < 0:
            # one-sided at a zero jitter (the likelihood is even in jitter)
            hp, lp = L(tp)
            h0, l0 = L(theta)
            g[i] = ((hp - h0) + (lp - l0)) / h
            continue
        hp, lp = L(tp)
        hm, lm = L(tm)
        g[i] = ((hp - hm) + (lp - lm)) / (tp[i] - tm[i])
    return g


def loglik_grad_inst_fd(ts, te, y, yerr, sigma, omega0, quality, jitter, instrument, amp, off, rel_step=1e-6,
                        kinds=None):
    """Central differences of the log-likelihood in the per-instrument
    amplitudes and offsets (Sec. 2.2 observation model with one amplitude a_i
    and offset c_i per instrument label).  Returns (d amp_0..I-1, d off_0..I-1).
    Offsets use an absolute step of rel_step * max(1, |c_i|)."""
    amp = np.asarray(amp, dtype=np.float64)
    off = np.asarray(off, dtype=np.float64)
    ni = len(amp)

    def L(a, c):
        ea, ec = expand_instruments(instrument, a, c)
        return loglik_hilo(ts, te, y, yerr, sigma, omega0, quality, jitter, kinds=kinds, amp=ea, off=ec)

    g = np.zeros(2 * ni)
    for i in range(2 * ni):
        base = amp if i < ni else off
        k = i % ni
        h = rel_step * abs(base[k]) if i < ni else rel_step * max(1.0, abs(base[k]))
        p = base.copy()
        m = base.copy()
        p[k] += h
        m[k] -= h
        if i < ni:
            hp, lp = L(p, off)
            hm, lm = L(m, off)
        else:
            hp, lp = L(amp, p)
            hm, lm = L(amp, m)
        g[i] = ((hp - hm) + (lp - lm)) / (p[k] - m[k])
    return g
