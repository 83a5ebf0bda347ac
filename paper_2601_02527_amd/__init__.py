"""Python binding of the gp_ssm HIP library (``libgp_ssm.so``).

Thin argument marshalling over the C-ABI declared in ``include/gp_ssm.h``:
every numerical step runs in the library's kernels.  PyTorch supplies device
memory and the current stream.  Importing this package does not need a GPU;
creating a plan or running a computation does, and raises if the library or
the device is missing.

    plan = Plan(offsets, t_start, t_end, y, yerr)          # once per dataset
    ll = plan.loglik(sigma, omega0, quality, jitter)        # [B]
    ll, g = plan.loglik_grad(sigma, omega0, quality, jitter)  # g: [B, 3M+1]
    ll = loglik_autograd(plan, sigma, omega0, quality, jitter)  # differentiable
    out = plan.smooth(sigma, omega0, quality, jitter, test_offsets, t_test)

    plan.set_term_kinds(["sho", "real"])                    # real exponential terms
    plan.set_instruments(labels, n_inst)                    # per-measurement labels
    ll, g = plan.loglik_grad_inst(sigma, omega0, quality, jitter, amp, off)
    ll = loglik_inst_autograd(plan, sigma, omega0, quality, jitter, amp, off)
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgp_ssm.so")

GP_SSM_OK = 0
TERM_SHO, TERM_REAL = 0, 1
TERM_CODES = {"sho": TERM_SHO, "real": TERM_REAL}
ERRORS = {-1: "EINVAL", -2: "EDATA", -3: "EPARAM", -4: "EOVERLAP", -5: "ENUMERIC", -6: "EDEVICE", -7: "ENOMEM"}

# every symbol include/gp_ssm.h declares
EXPORTS = [
    "gp_ssm_plan_default_options", "gp_ssm_plan_create", "gp_ssm_plan_destroy", "gp_ssm_plan_set_term_kinds",
    "gp_ssm_plan_set_instruments", "gp_ssm_plan_get_stats",
    "gp_ssm_plan_loglik", "gp_ssm_plan_loglik_noalloc", "gp_ssm_plan_loglik_grad", "gp_ssm_plan_loglik_inst",
    "gp_ssm_plan_loglik_grad_inst", "gp_ssm_plan_smooth", "gp_ssm_plan_smooth_terms", "gp_ssm_plan_smooth_inst",
    "gp_ssm_plan_plain_loglik", "gp_ssm_plan_loglik_sqrt",
    "gp_ssm_plan_loglik_sqrt_split", "gp_ssm_loglik", "gp_ssm_loglik_grad", "gp_ssm_smooth", "gp_ssm_autotune",
    "gp_ssm_autotune_candidates", "gp_ssm_profile_enable", "gp_ssm_profile_reset",
    "gp_ssm_profile_read", "gp_ssm_last_error", "gp_ssm_version",
]


class GpSsmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"gp_ssm error {ERRORS.get(code, code)}: {msg}")
        self.code = code


class PlanOptions(ctypes.Structure):
    _fields_ = [("chunk_min", ctypes.c_int32), ("chunk_target", ctypes.c_int32), ("target_chunks", ctypes.c_int64),
                ("single_chunk", ctypes.c_int32), ("threads", ctypes.c_int32), ("record_budget", ctypes.c_int64)]


class PlanStats(ctypes.Structure):
    _fields_ = [("n_series", ctypes.c_int64), ("n_meas", ctypes.c_int64), ("n_events", ctypes.c_int64),
                ("n_events_padded", ctypes.c_int64), ("n_chunks", ctypes.c_int32), ("n_segments", ctypes.c_int32),
                ("max_slots", ctypes.c_int32), ("max_chunk_len", ctypes.c_int32),
                ("device_bytes", ctypes.c_int64), ("record_bytes", ctypes.c_int64)]


_lib = None


def library():
    """Loads the library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2601_02527_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64
    L.gp_ssm_plan_default_options.argtypes = [ctypes.POINTER(PlanOptions)]
    L.gp_ssm_plan_default_options.restype = None
    L.gp_ssm_plan_create.argtypes = [i64, vp, vp, vp, vp, vp, ctypes.POINTER(PlanOptions), vp, ctypes.POINTER(vp)]
    L.gp_ssm_plan_destroy.argtypes = [vp]
    L.gp_ssm_plan_destroy.restype = None
    L.gp_ssm_plan_get_stats.argtypes = [vp, ctypes.POINTER(PlanStats)]
    L.gp_ssm_plan_set_term_kinds.argtypes = [vp, i32, ctypes.POINTER(i32)]
    L.gp_ssm_plan_set_instruments.argtypes = [vp, i32, vp, vp]
    L.gp_ssm_plan_loglik_inst.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp, vp, vp, vp]
    L.gp_ssm_plan_loglik_grad_inst.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
    L.gp_ssm_plan_smooth_inst.argtypes = [vp, i32] + [vp] * 17
    L.gp_ssm_plan_loglik.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp, vp]
    L.gp_ssm_plan_loglik_noalloc.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp, vp]
    L.gp_ssm_plan_loglik_grad.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp, vp, vp]
    L.gp_ssm_plan_smooth.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
    L.gp_ssm_plan_smooth_terms.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
    L.gp_ssm_plan_plain_loglik.argtypes = [vp, i64, i64, i32, vp, vp, vp, vp, vp, vp]
    L.gp_ssm_plan_loglik_sqrt.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp, vp, vp, vp]
    L.gp_ssm_plan_loglik_sqrt_split.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp, vp, vp, vp]
    L.gp_ssm_loglik.argtypes = [i64, vp, vp, vp, vp, vp, i32, vp, vp, vp, vp, vp, vp, vp]
    L.gp_ssm_loglik_grad.argtypes = [i64, vp, vp, vp, vp, vp, i32, vp, vp, vp, vp, vp, vp, vp, vp]
    L.gp_ssm_smooth.argtypes = [i64, vp, vp, vp, vp, vp, i32, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp]
    L.gp_ssm_autotune.argtypes = [i64, vp, vp, vp, vp, vp, i32, vp, vp, vp, vp, i32, ctypes.c_char_p,
                                  ctypes.POINTER(PlanOptions), ctypes.POINTER(ctypes.c_double), vp]
    L.gp_ssm_autotune_candidates.argtypes = [ctypes.POINTER(i64), i32]
    L.gp_ssm_profile_enable.argtypes = [i32]
    L.gp_ssm_profile_read.argtypes = [ctypes.POINTER(ctypes.c_char_p), ctypes.POINTER(i64),
                                      ctypes.POINTER(ctypes.c_double), i32]
    L.gp_ssm_last_error.restype = ctypes.c_char_p
    L.gp_ssm_version.restype = ctypes.c_char_p
    for name in ("gp_ssm_plan_create", "gp_ssm_plan_set_term_kinds", "gp_ssm_plan_set_instruments",
                 "gp_ssm_plan_get_stats", "gp_ssm_plan_loglik", "gp_ssm_plan_loglik_noalloc",
                 "gp_ssm_plan_loglik_grad", "gp_ssm_plan_loglik_inst", "gp_ssm_plan_loglik_grad_inst",
                 "gp_ssm_plan_smooth_inst",
                 "gp_ssm_plan_smooth", "gp_ssm_plan_smooth_terms", "gp_ssm_plan_plain_loglik", "gp_ssm_loglik",
                 "gp_ssm_loglik_grad",
                 "gp_ssm_smooth", "gp_ssm_autotune", "gp_ssm_autotune_candidates", "gp_ssm_profile_enable",
                 "gp_ssm_profile_reset", "gp_ssm_profile_read"):
        getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def _check(rc):
    if rc != 0:
        raise GpSsmError(rc, library().gp_ssm_last_error().decode())


def check_status(status):
    """Raises GpSsmError (EPARAM before ENUMERIC) if any series' status is not
    0; waits for the device."""
    st = status.cpu().numpy()
    for code in (-3, -5):
        bad = np.flatnonzero(st == code)
        if bad.size:
            raise GpSsmError(code, f"{bad.size} series (first {int(bad[0])})")
    bad = np.flatnonzero(st != 0)
    if bad.size:
        raise GpSsmError(int(st[bad[0]]), f"{bad.size} series (first {int(bad[0])})")


def _torch():
    import torch
    if not torch.cuda.is_available():
        raise RuntimeError("gp_ssm needs a GPU (torch.cuda.is_available() is False)")
    return torch


def _dev(x, dtype=None):
    """A contiguous device tensor (float64 unless dtype is given)."""
    torch = _torch()
    dtype = dtype or torch.float64
    if isinstance(x, torch.Tensor):
        return x.to(device="cuda", dtype=dtype).contiguous()
    return torch.as_tensor(np.ascontiguousarray(x), dtype=dtype, device="cuda")


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


def _stream():
    return ctypes.c_void_p(_torch().cuda.current_stream().cuda_stream)


def default_options(**kw):
    o = PlanOptions()
    library().gp_ssm_plan_default_options(ctypes.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


class Plan:
    """Hyperparameter-independent event plan of a batch of series."""

    def __init__(self, offsets, t_start, t_end, y, yerr, **options):
        torch = _torch()
        L = library()
        self.offsets = _dev(offsets, torch.int64)
        ts, te, yy, ye = (_dev(a) for a in (t_start, t_end, y, yerr))
        self.n_series = int(self.offsets.numel() - 1)
        self.n_meas = int(ts.numel())
        opt = default_options(**options)
        h = ctypes.c_void_p()
        _check(L.gp_ssm_plan_create(self.n_series, _ptr(self.offsets), _ptr(ts), _ptr(te), _ptr(yy), _ptr(ye),
                                    ctypes.byref(opt), _stream(), ctypes.byref(h)))
        self._h = h
        self.n_inst = 0

    def close(self):
        if getattr(self, "_h", None):
            library().gp_ssm_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def set_term_kinds(self, kinds):
        """Term kinds of later calls: a sequence of 'sho' / 'real' (or
        TERM_SHO / TERM_REAL); None for all SHO."""
        if kinds is None:
            _check(library().gp_ssm_plan_set_term_kinds(self._h, 0, None))
            return
        codes = [TERM_CODES.get(k, k) for k in kinds]
        arr = (ctypes.c_int32 * len(codes))(*codes)
        _check(library().gp_ssm_plan_set_term_kinds(self._h, len(codes), arr))

    def set_instruments(self, instrument, n_inst=None):
        """Instrument label of every measurement (int, 0..n_inst-1, in the
        plan's measurement order) for the per-instrument amplitude and offset
        of the *_inst calls; None removes the labels."""
        torch = _torch()
        if instrument is None:
            _check(library().gp_ssm_plan_set_instruments(self._h, 0, None, _stream()))
            self.n_inst = 0
            return
        lab = _dev(instrument, torch.int32).reshape(-1)
        if lab.numel() != self.n_meas:
            raise ValueError("one instrument label per measurement")
        ni = int(lab.max().item()) + 1 if n_inst is None else int(n_inst)
        _check(library().gp_ssm_plan_set_instruments(self._h, ni, _ptr(lab), _stream()))
        self.n_inst = ni

    def _inst(self, amp, off):
        # (without labels the library refuses the call)
        shape = (self.n_series, self.n_inst) if self.n_inst else (-1,)
        a = None if amp is None else _dev(amp).reshape(shape)
        c = None if off is None else _dev(off).reshape(shape)
        return a, c

    def loglik_inst(self, sigma, omega0, quality, jitter=None, amp=None, off=None, status=False, check=False):
        """Log-likelihood [B] with per-instrument amplitudes and offsets
        (amp, off: [B, n_inst]; None: 1 and 0)."""
        torch = _torch()
        M, s, w, q, j = self._params(sigma, omega0, quality, jitter)
        a, c = self._inst(amp, off)
        out = torch.empty(self.n_series, dtype=torch.float64, device="cuda")
        st = torch.empty(self.n_series, dtype=torch.int32, device="cuda")
        _check(library().gp_ssm_plan_loglik_inst(self._h, M, _ptr(s), _ptr(w), _ptr(q), _ptr(j), _ptr(a), _ptr(c),
                                                 _ptr(out), _ptr(st), _stream()))
        if check:
            check_status(st)
        return (out, st) if status else out

    def loglik_grad_inst(self, sigma, omega0, quality, jitter=None, amp=None, off=None, status=False, check=False):
        """Log-likelihood [B] and gradient [B, 3M+1+2 n_inst]: d/d sigma,
        omega0, Q, jitter, then amp_0..n_inst-1 and off_0..n_inst-1."""
        torch = _torch()
        M, s, w, q, j = self._params(sigma, omega0, quality, jitter)
        a, c = self._inst(amp, off)
        out = torch.empty(self.n_series, dtype=torch.float64, device="cuda")
        g = torch.empty(self.n_series, 3 * M + 1 + 2 * self.n_inst, dtype=torch.float64, device="cuda")
        st = torch.empty(self.n_series, dtype=torch.int32, device="cuda")
        _check(library().gp_ssm_plan_loglik_grad_inst(self._h, M, _ptr(s), _ptr(w), _ptr(q), _ptr(j), _ptr(a),
                                                      _ptr(c), _ptr(out), _ptr(g), _ptr(st), _stream()))
        if check:
            check_status(st)
        return (out, g, st) if status else (out, g)

    def stats(self):
        s = PlanStats()
        _check(library().gp_ssm_plan_get_stats(self._h, ctypes.byref(s)))
        return {f: getattr(s, f) for f, _ in PlanStats._fields_}

    def _params(self, sigma, omega0, quality, jitter):
        torch = _torch()
        sigma = _dev(sigma).reshape(self.n_series, -1)
        M = sigma.shape[1]
        omega0 = _dev(omega0).reshape(self.n_series, M)
        quality = _dev(quality).reshape(self.n_series, M)
        jit = None if jitter is None else _dev(jitter).reshape(self.n_series)
        return M, sigma, omega0, quality, jit

    def loglik(self, sigma, omega0, quality, jitter=None, status=False, check=False):
        """Log-likelihood of every series [B].  status=True also returns the
        per-series status; check=True waits and raises if any series failed
        (a failed series' outputs are NaN either way)."""
        torch = _torch()
        M, s, w, q, j = self._params(sigma, omega0, quality, jitter)
        out = torch.empty(self.n_series, dtype=torch.float64, device="cuda")
        st = torch.empty(self.n_series, dtype=torch.int32, device="cuda")
        _check(library().gp_ssm_plan_loglik(self._h, M, _ptr(s), _ptr(w), _ptr(q), _ptr(j), _ptr(out), _ptr(st),
                                            _stream()))
        if check:
            check_status(st)
        return (out, st) if status else out

    def loglik_noalloc(self, sigma, omega0, quality, jitter=None, out=None, status=None):
        """gp_ssm_plan_loglik_noalloc: the log-likelihood with the library's
        static workspace.  out [B] and status [B] (optional) are the caller's
        device tensors; this method allocates them only when not given."""
        torch = _torch()
        M, s, w, q, j = self._params(sigma, omega0, quality, jitter)
        if out is None:
            out = torch.empty(self.n_series, dtype=torch.float64, device="cuda")
        _check(library().gp_ssm_plan_loglik_noalloc(self._h, M, _ptr(s), _ptr(w), _ptr(q), _ptr(j), _ptr(out),
                                                    _ptr(status), _stream()))
        return out

    def loglik_grad(self, sigma, omega0, quality, jitter=None, status=False, check=False):
        """Log-likelihood [B] and gradient [B, 3M+1] (d/d sigma_1..M,
        omega0_1..M, Q_1..M, jitter); status and check as for loglik."""
        torch = _torch()
        M, s, w, q, j = self._params(sigma, omega0, quality, jitter)
        out = torch.empty(self.n_series, dtype=torch.float64, device="cuda")
        g = torch.empty(self.n_series, 3 * M + 1, dtype=torch.float64, device="cuda")
        st = torch.empty(self.n_series, dtype=torch.int32, device="cuda")
        _check(library().gp_ssm_plan_loglik_grad(self._h, M, _ptr(s), _ptr(w), _ptr(q), _ptr(j), _ptr(out), _ptr(g),
                                                 _ptr(st), _stream()))
        if check:
            check_status(st)
        return (out, g, st) if status else (out, g)

    def loglik_sqrt(self, sigma, omega0, quality, jitter=None, amp=None, off=None, status=False, check=False):
        """Log-likelihood [B] by the square-root (Cholesky-factor) filter,
        16 GPU lanes per series (gp_ssm_plan_loglik_sqrt); amp/off as for
        loglik_inst, status and check as for loglik."""
        torch = _torch()
        M, s, w, q, j = self._params(sigma, omega0, quality, jitter)
        a, c = self._inst(amp, off)
        out = torch.empty(self.n_series, dtype=torch.float64, device="cuda")
        st = torch.empty(self.n_series, dtype=torch.int32, device="cuda")
        _check(library().gp_ssm_plan_loglik_sqrt(self._h, M, _ptr(s), _ptr(w), _ptr(q), _ptr(j), _ptr(a), _ptr(c),
                                                 _ptr(out), _ptr(st), _stream()))
        if check:
            check_status(st)
        return (out, st) if status else out

    def loglik_sqrt_split(self, sigma, omega0, quality, jitter=None, amp=None, off=None, status=False, check=False):
        """Log-likelihood [B] by the square-root filter split in time at the
        plan's chunks (gp_ssm_plan_loglik_sqrt_split); arguments as for
        loglik_sqrt."""
        torch = _torch()
        M, s, w, q, j = self._params(sigma, omega0, quality, jitter)
        a, c = self._inst(amp, off)
        out = torch.empty(self.n_series, dtype=torch.float64, device="cuda")
        st = torch.empty(self.n_series, dtype=torch.int32, device="cuda")
        _check(library().gp_ssm_plan_loglik_sqrt_split(self._h, M, _ptr(s), _ptr(w), _ptr(q), _ptr(j), _ptr(a),
                                                       _ptr(c), _ptr(out), _ptr(st), _stream()))
        if check:
            check_status(st)
        return (out, st) if status else out

    def plain_loglik(self, sigma, omega0, quality, jitter=None, first=0, count=None):
        torch = _torch()
        M, s, w, q, j = self._params(sigma, omega0, quality, jitter)
        count = self.n_series - first if count is None else count
        out = torch.full((self.n_series,), float("nan"), dtype=torch.float64, device="cuda")
        _check(library().gp_ssm_plan_plain_loglik(self._h, first, count, M, _ptr(s), _ptr(w), _ptr(q), _ptr(j),
                                                  _ptr(out), _stream()))
        return out

    def smooth(self, sigma, omega0, quality, jitter, test_offsets, t_test, data=True, terms=False, amp=None,
               off=None):
        """Posterior at the data and at the test times; with terms=True also
        each term's latent posterior at the test times (term_mean, term_var:
        [n_test, M]).  amp, off ([B, n_inst], after set_instruments): the
        per-instrument amplitudes and offsets; mean_data/var_data are then
        those of the noise-free measured quantity."""
        torch = _torch()
        M, s, w, q, j = self._params(sigma, omega0, quality, jitter)
        to = _dev(test_offsets, torch.int64)
        tt = _dev(t_test)
        mt = torch.empty_like(tt)
        vt = torch.empty_like(tt)
        md = torch.empty(self.n_meas, dtype=torch.float64, device="cuda") if data else None
        vd = torch.empty(self.n_meas, dtype=torch.float64, device="cuda") if data else None
        ll = torch.empty(self.n_series, dtype=torch.float64, device="cuda")
        st = torch.empty(self.n_series, dtype=torch.int32, device="cuda")
        out = dict(mean_test=mt, var_test=vt, mean_data=md, var_data=vd, loglik=ll, status=st)
        if amp is not None or off is not None:
            a, c = self._inst(amp, off)
            tm = tv = None
            if terms:
                tm = torch.empty((tt.numel(), M), dtype=torch.float64, device="cuda")
                tv = torch.empty_like(tm)
                out.update(term_mean=tm, term_var=tv)
            _check(library().gp_ssm_plan_smooth_inst(self._h, M, _ptr(s), _ptr(w), _ptr(q), _ptr(j), _ptr(a), _ptr(c),
                                                     _ptr(to), _ptr(tt), _ptr(mt), _ptr(vt), _ptr(tm), _ptr(tv),
                                                     _ptr(md), _ptr(vd), _ptr(ll), _ptr(st), _stream()))
        elif terms:
            tm = torch.empty((tt.numel(), M), dtype=torch.float64, device="cuda")
            tv = torch.empty_like(tm)
            _check(library().gp_ssm_plan_smooth_terms(self._h, M, _ptr(s), _ptr(w), _ptr(q), _ptr(j), _ptr(to),
                                                      _ptr(tt), _ptr(mt), _ptr(vt), _ptr(tm), _ptr(tv), _ptr(md),
                                                      _ptr(vd), _ptr(ll), _ptr(st), _stream()))
            out.update(term_mean=tm, term_var=tv)
        else:
            _check(library().gp_ssm_plan_smooth(self._h, M, _ptr(s), _ptr(w), _ptr(q), _ptr(j), _ptr(to), _ptr(tt),
                                                _ptr(mt), _ptr(vt), _ptr(md), _ptr(vd), _ptr(ll), _ptr(st), _stream()))
        return out


def _one_shot_inputs(offsets, t_start, t_end, y, yerr, sigma, omega0, quality, jitter):
    torch = _torch()
    off = _dev(offsets, torch.int64)
    B = off.numel() - 1
    sigma = _dev(sigma).reshape(B, -1)
    M = sigma.shape[1]
    arrs = [_dev(a) for a in (t_start, t_end, y, yerr)]
    omega0 = _dev(omega0).reshape(B, M)
    quality = _dev(quality).reshape(B, M)
    jit = None if jitter is None else _dev(jitter).reshape(B)
    return B, M, off, arrs, sigma, omega0, quality, jit


def loglik(offsets, t_start, t_end, y, yerr, sigma, omega0, quality, jitter=None):
    """One-shot log-likelihood (gp_ssm_loglik: plan, run, destroy)."""
    torch = _torch()
    B, M, off, (ts, te, yy, ye), s, w, q, j = _one_shot_inputs(offsets, t_start, t_end, y, yerr, sigma, omega0,
                                                               quality, jitter)
    ll = torch.empty(B, dtype=torch.float64, device="cuda")
    _check(library().gp_ssm_loglik(B, _ptr(off), _ptr(ts), _ptr(te), _ptr(yy), _ptr(ye), M, _ptr(s), _ptr(w), _ptr(q),
                                   _ptr(j), _ptr(ll), None, _stream()))
    return ll


def loglik_grad(offsets, t_start, t_end, y, yerr, sigma, omega0, quality, jitter=None):
    """One-shot log-likelihood and gradient (gp_ssm_loglik_grad)."""
    torch = _torch()
    B, M, off, (ts, te, yy, ye), s, w, q, j = _one_shot_inputs(offsets, t_start, t_end, y, yerr, sigma, omega0,
                                                               quality, jitter)
    ll = torch.empty(B, dtype=torch.float64, device="cuda")
    g = torch.empty((B, 3 * M + 1), dtype=torch.float64, device="cuda")
    _check(library().gp_ssm_loglik_grad(B, _ptr(off), _ptr(ts), _ptr(te), _ptr(yy), _ptr(ye), M, _ptr(s), _ptr(w),
                                        _ptr(q), _ptr(j), _ptr(ll), _ptr(g), None, _stream()))
    return ll, g


def smooth(offsets, t_start, t_end, y, yerr, sigma, omega0, quality, jitter, test_offsets, t_test, data=True):
    """One-shot posterior (gp_ssm_smooth)."""
    torch = _torch()
    B, M, off, (ts, te, yy, ye), s, w, q, j = _one_shot_inputs(offsets, t_start, t_end, y, yerr, sigma, omega0,
                                                               quality, jitter)
    to = _dev(test_offsets, torch.int64)
    tt = _dev(t_test)
    mt, vt = torch.empty_like(tt), torch.empty_like(tt)
    md = torch.empty(ts.numel(), dtype=torch.float64, device="cuda") if data else None
    vd = torch.empty(ts.numel(), dtype=torch.float64, device="cuda") if data else None
    st = torch.empty(B, dtype=torch.int32, device="cuda")
    _check(library().gp_ssm_smooth(B, _ptr(off), _ptr(ts), _ptr(te), _ptr(yy), _ptr(ye), M, _ptr(s), _ptr(w), _ptr(q),
                                   _ptr(j), _ptr(to), _ptr(tt), _ptr(mt), _ptr(vt), _ptr(md), _ptr(vd), _ptr(st),
                                   _stream()))
    return dict(mean_test=mt, var_test=vt, mean_data=md, var_data=vd, status=st)


def _autograd_function():
    torch = _torch()

    class LogLikelihood(torch.autograd.Function):
        """log-likelihood per series with its gradient from the adjoint kernel."""

        @staticmethod
        def forward(ctx, sigma, omega0, quality, jitter, plan):
            need = any(ctx.needs_input_grad[:4])
            if need:
                ll, g = plan.loglik_grad(sigma, omega0, quality, jitter)
                ctx.save_for_backward(g)
                ctx.M = sigma.reshape(plan.n_series, -1).shape[1]
                ctx.shapes = (sigma.shape, omega0.shape, quality.shape, None if jitter is None else jitter.shape)
            else:
                ll = plan.loglik(sigma, omega0, quality, jitter)
            return ll

        @staticmethod
        def backward(ctx, gout):
            (g,) = ctx.saved_tensors
            M = ctx.M
            gg = g * gout[:, None]
            ds = gg[:, :M].reshape(ctx.shapes[0])
            dw = gg[:, M:2 * M].reshape(ctx.shapes[1])
            dq = gg[:, 2 * M:3 * M].reshape(ctx.shapes[2])
            dj = None if ctx.shapes[3] is None else gg[:, 3 * M].reshape(ctx.shapes[3])
            return ds, dw, dq, dj, None

    return LogLikelihood


def _autograd_inst_function():
    torch = _torch()

    class LogLikelihoodInst(torch.autograd.Function):
        """log-likelihood per series with per-instrument amplitudes and
        offsets, and its gradient from the adjoint kernel."""

        @staticmethod
        def forward(ctx, sigma, omega0, quality, jitter, amp, off, plan):
            ll, g = plan.loglik_grad_inst(sigma, omega0, quality, jitter, amp, off)
            ctx.save_for_backward(g)
            ctx.M = sigma.reshape(plan.n_series, -1).shape[1]
            ctx.ni = plan.n_inst
            ctx.shapes = (sigma.shape, omega0.shape, quality.shape, None if jitter is None else jitter.shape,
                          None if amp is None else amp.shape, None if off is None else off.shape)
            return ll

        @staticmethod
        def backward(ctx, gout):
            (g,) = ctx.saved_tensors
            M, ni, sh = ctx.M, ctx.ni, ctx.shapes
            gg = g * gout[:, None]
            ds = gg[:, :M].reshape(sh[0])
            dw = gg[:, M:2 * M].reshape(sh[1])
            dq = gg[:, 2 * M:3 * M].reshape(sh[2])
            dj = None if sh[3] is None else gg[:, 3 * M].reshape(sh[3])
            k = 3 * M + 1
            da = None if sh[4] is None else gg[:, k:k + ni].reshape(sh[4])
            dc = None if sh[5] is None else gg[:, k + ni:k + 2 * ni].reshape(sh[5])
            return ds, dw, dq, dj, da, dc, None

    return LogLikelihoodInst


_LL = None
_LLI = None


def loglik_autograd(plan, sigma, omega0, quality, jitter=None):
    """Differentiable log-likelihood of every series of ``plan``."""
    global _LL
    if _LL is None:
        _LL = _autograd_function()
    return _LL.apply(sigma, omega0, quality, jitter, plan)


def loglik_inst_autograd(plan, sigma, omega0, quality, jitter=None, amp=None, off=None):
    """Differentiable log-likelihood with per-instrument amplitudes and
    offsets ([B, n_inst] tensors, after plan.set_instruments)."""
    global _LLI
    if _LLI is None:
        _LLI = _autograd_inst_function()
    return _LLI.apply(sigma, omega0, quality, jitter, amp, off, plan)


def autotune_candidates():
    """The target chunk counts the autotuner tries."""
    n = library().gp_ssm_autotune_candidates(None, 0)
    buf = (ctypes.c_int64 * n)()
    library().gp_ssm_autotune_candidates(buf, n)
    return list(buf)


def default_cache_path():
    """Where the autotuner's choices are kept unless told otherwise."""
    base = os.environ.get("XDG_CACHE_HOME") or os.path.join(os.path.expanduser("~"), ".cache")
    return os.path.join(base, "gp_ssm", "autotune.txt")


def autotune(offsets, t_start, t_end, y, yerr, sigma, omega0, quality, jitter=None, grad=True, cache=None):
    """gp_ssm_autotune: plan options (a dict for Plan(**options)) with the
    fastest target chunk count for this workload, and its time per call in
    ms.  cache: a file path, False for none, or None for default_cache_path()."""
    B, M, off, (ts, te, yy, ye), s, w, q, j = _one_shot_inputs(offsets, t_start, t_end, y, yerr, sigma, omega0,
                                                               quality, jitter)
    if cache is None:
        cache = default_cache_path()
        os.makedirs(os.path.dirname(cache), exist_ok=True)
    best = PlanOptions()
    ms = ctypes.c_double()
    _check(library().gp_ssm_autotune(B, _ptr(off), _ptr(ts), _ptr(te), _ptr(yy), _ptr(ye), M, _ptr(s), _ptr(w),
                                     _ptr(q), _ptr(j), 1 if grad else 0, cache.encode() if cache else None,
                                     ctypes.byref(best), ctypes.byref(ms), _stream()))
    return {f: getattr(best, f) for f, _ in PlanOptions._fields_}, ms.value


def profile_enable(on=True):
    _check(library().gp_ssm_profile_enable(1 if on else 0))


def profile_reset():
    _check(library().gp_ssm_profile_reset())


def profile_read():
    L = library()
    cap = 64
    names = (ctypes.c_char_p * cap)()
    counts = (ctypes.c_int64 * cap)()
    tot = (ctypes.c_double * cap)()
    n = L.gp_ssm_profile_read(names, counts, tot, cap)
    return {names[i].decode(): (int(counts[i]), float(tot[i])) for i in range(min(n, cap))}


def version():
    return library().gp_ssm_version().decode()
