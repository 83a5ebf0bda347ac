"""GPU parity for the observation model with one amplitude a_i and one
offset c_i per instrument (gp_ssm_plan_set_instruments and the *_inst entry
points): log-likelihood, gradient (sigma, omega0, Q, jitter, then every a_i
and c_i) and smoother against the oracle, with SHO terms and with a real
term; the entry points without amplitudes on a labelled plan; validation of
amplitudes, offsets and labels; host-memory amplitudes through the C-ABI.

Tolerances as in test_gpu_parity: log-likelihood 1e-9 relative, gradient
1e-6 (relative to max(|g_i|, 1e-3 max|g|)), smoothed moments 1e-9 of the
prior standard deviation / variance (times the amplitude for the data)."""
import ctypes
import math

import numpy as np
import pytest

import workloads as W
from oracle import dense, kalman

pytestmark = pytest.mark.gpu

OPTS = (dict(chunk_min=1, chunk_target=1), dict(chunk_min=4, chunk_target=9), dict())


def _args(s):
    return (s["ts"], s["te"], s["y"], s["yerr"], s["sigma"], s["omega0"], s["quality"], s["jitter"])


def _grad_err(g, ref):
    den = np.maximum(np.abs(ref), 1e-3 * np.max(np.abs(ref)))
    return np.max(np.abs(g - ref) / den)


def _case(seed, M=2, ni=3, B=5, n_lo=10, n_hi=80):
    b = W.random_small_batch(seed, B=B, n_lo=n_lo, n_hi=n_hi, M=M, J=3)
    rng = np.random.default_rng(seed + 1000)
    lab = rng.integers(0, ni, len(b.t_start)).astype(np.int32)
    amp = rng.uniform(0.5, 1.8, (B, ni))
    off = rng.normal(0.0, 0.4, (B, ni))
    return b, lab, amp, off


def _series_inst(b, lab, amp, off, i):
    """Per-measurement amplitude and offset of series i, and its labels."""
    lo, hi = int(b.offsets[i]), int(b.offsets[i + 1])
    li = lab[lo:hi]
    a_n, c_n = kalman.expand_instruments(li, amp[i], off[i])
    return li, a_n, c_n


@pytest.mark.parametrize("kinds", [None, ["sho", "real"]])
def test_instruments_match_oracle(lib, kinds):
    b, lab, amp, off = _case(710 if kinds is None else 711)
    ni = amp.shape[1]
    ref = []
    for i in range(b.n_series):
        _, a_n, c_n = _series_inst(b, lab, amp, off, i)
        ref.append(kalman.loglik(*_args(b.series(i)), kinds=kinds, amp=a_n, off=c_n))
    ref = np.array(ref)
    for opt in OPTS:
        plan = lib.Plan(b.offsets, b.t_start, b.t_end, b.y, b.yerr, **opt)
        if kinds:
            plan.set_term_kinds(kinds)
        plan.set_instruments(lab, ni)
        ll, st = plan.loglik_inst(b.sigma, b.omega0, b.quality, b.jitter, amp, off, status=True)
        ll2, g, st2 = plan.loglik_grad_inst(b.sigma, b.omega0, b.quality, b.jitter, amp, off, status=True)
        ll, ll2, g = ll.cpu().numpy(), ll2.cpu().numpy(), g.cpu().numpy()
        assert np.all(st.cpu().numpy() == 0) and np.all(st2.cpu().numpy() == 0)
        assert g.shape == (b.n_series, 3 * b.n_terms + 1 + 2 * ni)
        rel = max(np.max(np.abs(ll - ref) / np.abs(ref)), np.max(np.abs(ll2 - ref) / np.abs(ref)))
        print(kinds, opt, rel)
        assert rel < 1e-9
    for i in (0, 2):
        s = b.series(i)
        li, a_n, c_n = _series_inst(b, lab, amp, off, i)
        gt = kalman.loglik_grad_fd(*_args(s), kinds=kinds, amp=a_n, off=c_n)
        gi = kalman.loglik_grad_inst_fd(*_args(s), li, amp[i], off[i], kinds=kinds)
        gfd = np.concatenate([gt, gi])
        # an instrument without measurements in this series has zero derivatives
        for k in range(ni):
            if not np.any(li == k):
                assert g[i][3 * b.n_terms + 1 + k] == 0.0 and g[i][3 * b.n_terms + 1 + ni + k] == 0.0
        e = _grad_err(g[i], gfd)
        print("gradient", i, e)
        assert e < 1e-6, (i, g[i], gfd)


def test_instrument_gradient_matches_dense(lib):
    """Against the dense oracle's analytic gradient (A K A + noise, Sec. 2.2)."""
    b, lab, amp, off = _case(712, B=2, n_lo=40, n_hi=60)
    ni = amp.shape[1]
    plan = lib.Plan(b.offsets, b.t_start, b.t_end, b.y, b.yerr, chunk_min=4, chunk_target=8)
    plan.set_instruments(lab, ni)
    ll, g = plan.loglik_grad_inst(b.sigma, b.omega0, b.quality, b.jitter, amp, off)
    ll, g = ll.cpu().numpy(), g.cpu().numpy()
    for i in range(b.n_series):
        li, _, _ = _series_inst(b, lab, amp, off, i)
        L, gd = dense.loglik_grad(*_args(b.series(i)), instrument=li, amp=amp[i], off=off[i])
        assert abs(ll[i] - L) < 1e-9 * abs(L)
        e = _grad_err(g[i], gd)
        print(i, e)
        assert e < 1e-6


def test_labelled_plan_without_amplitudes_is_the_plain_model(lib):
    b, lab, amp, off = _case(713)
    plain = lib.Plan(b.offsets, b.t_start, b.t_end, b.y, b.yerr)
    l0, g0 = (x.cpu().numpy() for x in plain.loglik_grad(b.sigma, b.omega0, b.quality, b.jitter))
    plan = lib.Plan(b.offsets, b.t_start, b.t_end, b.y, b.yerr)
    plan.set_instruments(lab, 3)
    l1, g1 = (x.cpu().numpy() for x in plan.loglik_grad(b.sigma, b.omega0, b.quality, b.jitter))
    l2 = plan.loglik_inst(b.sigma, b.omega0, b.quality, b.jitter).cpu().numpy()
    l3, g3 = (x.cpu().numpy() for x in plan.loglik_grad_inst(b.sigma, b.omega0, b.quality, b.jitter,
                                                              np.ones((b.n_series, 3)), np.zeros((b.n_series, 3))))
    assert g1.shape == g0.shape and g3.shape == (b.n_series, g0.shape[1] + 6)
    for l in (l1, l2, l3):
        assert np.all(np.abs(l - l0) <= 1e-12 * np.abs(l0))
    assert _grad_err(g1, g0) < 1e-10 and _grad_err(g3[:, :g0.shape[1]], g0) < 1e-10
    # removing the labels goes back to the plain kernels
    plan.set_instruments(None)
    l4 = plan.loglik(b.sigma, b.omega0, b.quality, b.jitter).cpu().numpy()
    assert np.all(np.abs(l4 - l0) <= 1e-12 * np.abs(l0))
    with pytest.raises(lib.GpSsmError):
        plan.loglik_grad_inst(b.sigma, b.omega0, b.quality, b.jitter, amp, off)


def test_instrument_smoother_matches_oracle(lib):
    b, lab, amp, off = _case(714)
    ni = amp.shape[1]
    nt = 11
    tt = np.concatenate([np.linspace(b.series(i)["ts"].min() - 0.05, b.series(i)["te"].max() + 0.05, nt)
                         for i in range(b.n_series)])
    to = np.arange(b.n_series + 1, dtype=np.int64) * nt
    for opt in (dict(chunk_min=4, chunk_target=8), dict()):
        plan = lib.Plan(b.offsets, b.t_start, b.t_end, b.y, b.yerr, **opt)
        plan.set_instruments(lab, ni)
        o = plan.smooth(b.sigma, b.omega0, b.quality, b.jitter, to, tt, terms=True, amp=amp, off=off)
        o = {k: v.cpu().numpy() for k, v in o.items() if v is not None}
        assert np.all(o["status"] == 0)
        for i in range(b.n_series):
            s = b.series(i)
            _, a_n, c_n = _series_inst(b, lab, amp, off, i)
            L, mt, vt, md, vd, tm, tv = kalman.smooth(*_args(s), t_test=tt[to[i]:to[i + 1]], terms=True, amp=a_n,
                                                      off=c_n)
            k0 = float(np.sum(np.asarray(s["sigma"]) ** 2))
            lo, hi = int(b.offsets[i]), int(b.offsets[i + 1])
            amax = float(np.max(amp[i]))
            errs = (abs(o["loglik"][i] - L) / abs(L),
                    np.max(np.abs(o["mean_data"][lo:hi] - md)) / (amax * math.sqrt(k0)),
                    np.max(np.abs(o["var_data"][lo:hi] - vd)) / (amax * amax * k0),
                    np.max(np.abs(o["mean_test"][to[i]:to[i + 1]] - mt)) / math.sqrt(k0),
                    np.max(np.abs(o["var_test"][to[i]:to[i + 1]] - vt)) / k0,
                    np.max(np.abs(o["term_mean"][to[i]:to[i + 1]] - tm)) / math.sqrt(k0),
                    np.max(np.abs(o["term_var"][to[i]:to[i + 1]] - tv)) / k0)
            print(opt, i, errs)
            assert max(errs) < 1e-9, (opt, i, errs)


def test_instrument_validation(lib):
    import torch
    b, lab, amp, off = _case(715)
    plan = lib.Plan(b.offsets, b.t_start, b.t_end, b.y, b.yerr)
    bad = lab.copy()
    bad[5] = 3
    with pytest.raises(lib.GpSsmError):
        plan.set_instruments(bad, 3)
    with pytest.raises(lib.GpSsmError):
        plan.set_instruments(lab, 9)  # above the maximum number of instruments
    with pytest.raises(lib.GpSsmError):  # no labels yet
        plan.loglik_inst(b.sigma, b.omega0, b.quality, b.jitter, amp, off)
    plan.set_instruments(lab, 3)
    good = plan.loglik_inst(b.sigma, b.omega0, b.quality, b.jitter, amp, off).cpu().numpy()
    for k, v in (("amp", 0.0), ("amp", -1.0), ("amp", np.nan), ("amp", np.inf), ("off", np.nan), ("off", np.inf)):
        a2, c2 = amp.copy(), off.copy()
        (a2 if k == "amp" else c2)[1, 2] = v
        ll, st = plan.loglik_inst(b.sigma, b.omega0, b.quality, b.jitter, a2, c2, status=True)
        ll, g, st2 = plan.loglik_grad_inst(b.sigma, b.omega0, b.quality, b.jitter, a2, c2, status=True)
        ll, st, st2, g = ll.cpu().numpy(), st.cpu().numpy(), st2.cpu().numpy(), g.cpu().numpy()
        assert st[1] == -3 and st2[1] == st[1]
        assert np.isnan(ll[1]) and np.all(np.isnan(g[1]))
        others = [i for i in range(b.n_series) if i != 1]
        assert np.all(st[others] == 0) and np.all(ll[others] == good[others])
        with pytest.raises(lib.GpSsmError):
            plan.loglik_inst(b.sigma, b.omega0, b.quality, b.jitter, a2, c2, check=True)


def test_instrument_parameters_from_host_memory(lib):
    """amp and off in host memory through the C-ABI (staged on the stream)."""
    import torch
    b, lab, amp, off = _case(716)
    plan = lib.Plan(b.offsets, b.t_start, b.t_end, b.y, b.yerr)
    plan.set_instruments(torch.as_tensor(lab, device="cuda"), 3)
    ref = plan.loglik_inst(b.sigma, b.omega0, b.quality, b.jitter, amp, off).cpu().numpy()
    M = b.n_terms
    hs = [np.ascontiguousarray(a, dtype=np.float64) for a in (b.sigma, b.omega0, b.quality, b.jitter, amp, off)]
    hp = [h.ctypes.data_as(ctypes.c_void_p) for h in hs]
    out = torch.empty(b.n_series, dtype=torch.float64, device="cuda")
    rc = lib.library().gp_ssm_plan_loglik_inst(plan._h, M, *hp, ctypes.c_void_p(out.data_ptr()), None, None)
    assert rc == 0
    torch.cuda.synchronize()
    assert np.all(out.cpu().numpy() == ref)


def test_instrument_autograd_function(lib):
    """loglik_inst_autograd: the library's gradient reaches every input
    (hyperparameters, amplitudes, offsets), scaled by the upstream weights."""
    import torch
    b, lab, amp, off = _case(717, B=3)
    plan = lib.Plan(b.offsets, b.t_start, b.t_end, b.y, b.yerr)
    plan.set_instruments(lab, 3)
    t = [torch.tensor(a, device="cuda", requires_grad=True) for a in (b.sigma, b.omega0, b.quality, b.jitter, amp, off)]
    ll = lib.loglik_inst_autograd(plan, *t)
    wts = torch.tensor([1.0, -2.0, 0.5], dtype=torch.float64, device="cuda")
    (ll * wts).sum().backward()
    _, g = plan.loglik_grad_inst(b.sigma, b.omega0, b.quality, b.jitter, amp, off)
    g = g.cpu().numpy() * np.array([1.0, -2.0, 0.5])[:, None]
    M = b.n_terms
    cols = [slice(0, M), slice(M, 2 * M), slice(2 * M, 3 * M), 3 * M, slice(3 * M + 1, 3 * M + 4),
            slice(3 * M + 4, 3 * M + 7)]
    for x, c in zip(t, cols):
        assert np.allclose(x.grad.cpu().numpy(), g[:, c], rtol=1e-14, atol=0)
