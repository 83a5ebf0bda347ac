"""GPU parity at the benchmark's full sizes, in the launch configuration that
bench.py times (same workload generators, default plan options): sampled
outputs against the oracle where it can compute them one by one, and for the
1e7-point series, whose oracle would take minutes, properties that hold at any
size (the same result from two scan structures).

Tolerances as in test_gpu_parity (log-likelihood 1e-9 relative, gradient 1e-6),
and for the smoother the oracle's own accuracy at this size (see its test).
"""
import gc

import numpy as np
import pytest

import workloads as W
from oracle import kalman

pytestmark = pytest.mark.gpu

LL_TOL = 1e-9
GRAD_TOL = 1e-6


def _args(s):
    return (s["ts"], s["te"], s["y"], s["yerr"], s["sigma"], s["omega0"], s["quality"], s["jitter"])


def _grad_err(g, ref):
    den = np.maximum(np.abs(ref), 1e-3 * np.max(np.abs(ref)))
    return np.max(np.abs(g - ref) / den)


def _free():
    import torch
    gc.collect()
    torch.cuda.empty_cache()


def _sampled_checks(lib, b, sample, fd_series):
    plan = lib.Plan(b.offsets, b.t_start, b.t_end, b.y, b.yerr)
    ll, g = plan.loglik_grad(b.sigma, b.omega0, b.quality, b.jitter)
    ll1 = plan.loglik(b.sigma, b.omega0, b.quality, b.jitter)
    ll, g, ll1 = ll.cpu().numpy(), g.cpu().numpy(), ll1.cpu().numpy()
    assert np.all(np.isfinite(ll)) and np.all(np.isfinite(g))
    assert np.array_equal(ll, ll1) or np.max(np.abs(ll - ll1) / np.abs(ll1)) < 1e-13
    for i in sample:
        s = b.series(int(i))
        ref = kalman.loglik(*_args(s))
        rel = abs(ll[i] - ref) / abs(ref)
        print("series", i, "points", len(s["ts"]), "rel", rel)
        assert rel < LL_TOL, (i, rel)
    s = b.series(int(fd_series))
    gref = kalman.loglik_grad_fd(*_args(s))
    gs = g[fd_series]
    if s["jitter"] == 0.0:
        # the likelihood depends on the jitter through its square: the
        # derivative at zero is exactly 0, where a difference quotient, one
        # sided at the boundary, is not
        assert gs[-1] == 0.0
        gs, gref = gs[:-1], gref[:-1]
    e = _grad_err(gs, gref)
    print("gradient of series", fd_series, "err", e)
    assert e < GRAD_TOL, e
    del plan


def test_grad_1024_sampled(lib):
    """1024 series x 1e4 exposures, 3 terms + jitter, up to 3 overlapping."""
    b = W.grad_1024()
    _sampled_checks(lib, b, sample=[0, 511, 1023], fd_series=511)
    _free()


def test_grad_1024_instruments_sampled(lib):
    """The gradient batch with three instrument labels per series and their
    amplitudes and offsets, drawn as bench.py draws them for its
    with_instruments timing: sampled series' log-likelihood and one series'
    full gradient (hyperparameters, amplitudes, offsets) against the oracle."""
    b = W.grad_1024()
    B, points = b.n_series, int(b.offsets[-1])
    rng = np.random.default_rng(7)
    ni = 3
    lab = rng.integers(0, ni, points).astype(np.int32)
    amp, off = rng.uniform(0.8, 1.2, (B, ni)), rng.normal(0.0, 0.1, (B, ni))
    plan = lib.Plan(b.offsets, b.t_start, b.t_end, b.y, b.yerr)
    plan.set_instruments(lab, ni)
    ll, g = plan.loglik_grad_inst(b.sigma, b.omega0, b.quality, b.jitter, amp, off)
    ll, g = ll.cpu().numpy(), g.cpu().numpy()
    assert np.all(np.isfinite(ll)) and np.all(np.isfinite(g)) and g.shape == (B, 3 * b.n_terms + 1 + 2 * ni)
    for i in (0, 700, 1023):
        s = b.series(i)
        lo, hi = int(b.offsets[i]), int(b.offsets[i + 1])
        a_n, c_n = kalman.expand_instruments(lab[lo:hi], amp[i], off[i])
        ref = kalman.loglik(*_args(s), amp=a_n, off=c_n)
        rel = abs(ll[i] - ref) / abs(ref)
        print("series", i, "rel", rel)
        assert rel < LL_TOL, (i, rel)
    i = 700
    s = b.series(i)
    lo, hi = int(b.offsets[i]), int(b.offsets[i + 1])
    a_n, c_n = kalman.expand_instruments(lab[lo:hi], amp[i], off[i])
    gref = np.concatenate([kalman.loglik_grad_fd(*_args(s), amp=a_n, off=c_n),
                           kalman.loglik_grad_inst_fd(*_args(s), lab[lo:hi], amp[i], off[i])])
    e = _grad_err(g[i], gref)
    print("gradient of series", i, "err", e)
    assert e < GRAD_TOL, e
    del plan
    _free()


def test_batch_4096_sampled(lib):
    """4096 series of 1e3-5e4 exposures: the shortest, a median and the
    longest series against the oracle, the shortest's gradient against finite
    differences."""
    b = W.batch_4096()
    n = np.diff(np.asarray(b.offsets))
    order = np.argsort(n, kind="stable")
    sample = [order[0], order[len(order) // 2], order[-1]]
    _sampled_checks(lib, b, sample=sample, fd_series=order[0])
    _free()


def test_long_1e7_two_scan_structures(lib):
    """One series of 1e7 exposures: the default plan (2043 segments, a second
    scan level over groups of 64) and a plan with at most 64 segments (one
    scan level, long chunks) give the same log-likelihood and gradient."""
    b = W.long_1e7()
    p0 = lib.Plan(b.offsets, b.t_start, b.t_end, b.y, b.yerr)
    s0 = p0.stats()
    ll0, g0 = p0.loglik_grad(b.sigma, b.omega0, b.quality, b.jitter)
    ll0, g0 = ll0.cpu().numpy(), g0.cpu().numpy()
    del p0
    _free()
    n_ev = s0["n_events"]
    p1 = lib.Plan(b.offsets, b.t_start, b.t_end, b.y, b.yerr, chunk_target=-(-n_ev // (64 * 60)))
    s1 = p1.stats()
    ll1, g1 = p1.loglik_grad(b.sigma, b.omega0, b.quality, b.jitter)
    ll1, g1 = ll1.cpu().numpy(), g1.cpu().numpy()
    del p1
    _free()
    print(s0, s1, ll0, ll1, _grad_err(g0[0], g1[0]))
    assert s0["n_segments"] > 64 and s1["n_segments"] <= 64
    assert np.isfinite(ll0[0]) and np.all(np.isfinite(g0))
    assert abs(ll0[0] - ll1[0]) / abs(ll1[0]) < LL_TOL
    assert _grad_err(g0[0], g1[0]) < GRAD_TOL
    # the first 1e6 exposures: the scan (default plan) against the plain
    # sequential filter of the same series, one lane, no time splitting
    n = 1_000_000
    p2 = lib.Plan(np.array([0, n], dtype=np.int64), b.t_start[:n], b.t_end[:n], b.y[:n], b.yerr[:n])
    l_scan = p2.loglik(b.sigma, b.omega0, b.quality, b.jitter).cpu().numpy()
    l_plain = p2.plain_loglik(b.sigma, b.omega0, b.quality, b.jitter).cpu().numpy()
    print("1e6 prefix", p2.stats(), l_scan, l_plain)
    assert p2.stats()["n_segments"] > 64
    assert abs(l_scan[0] - l_plain[0]) / abs(l_plain[0]) < LL_TOL
    del p2
    _free()


def test_long_1e7_smoother(lib):
    """The smoother on the 1e7-exposure series (bench.py's C5 smoother call:
    every measurement and 1e4 test times): the default plan and a plan with
    at most 64 segments agree (means within 1e-9 of the prior standard
    deviation, variances within 1e-9 of the prior variance), and properties
    that hold at any size: every posterior variance at a measurement lies in
    [0, yerr^2] (conditioning on more data than the measurement itself cannot
    raise it above R), every test-time variance in [0, prior variance]."""
    b = W.long_1e7()
    t_test = np.linspace(float(b.t_start[0]), float(b.t_end[-1]), 10_000)
    to = np.array([0, len(t_test)], dtype=np.int64)
    k0 = float(np.sum(np.asarray(b.sigma) ** 2))
    outs = []
    for opt in (dict(), dict(chunk_target=-(-2 * int(b.offsets[-1]) // (64 * 60)))):
        plan = lib.Plan(b.offsets, b.t_start, b.t_end, b.y, b.yerr, **opt)
        o = plan.smooth(b.sigma, b.omega0, b.quality, b.jitter, to, t_test)
        outs.append({k: o[k].cpu().numpy() for k in ("mean_data", "var_data", "mean_test", "var_test", "status")})
        print(opt, plan.stats())
        del plan, o
        _free()
    a, c = outs
    assert np.all(a["status"] == 0) and np.all(c["status"] == 0)
    R = np.asarray(b.yerr) ** 2 + float(b.jitter[0]) ** 2
    for o in outs:
        for k in ("mean_data", "var_data", "mean_test", "var_test"):
            assert np.all(np.isfinite(o[k])), k
        assert np.all(o["var_data"] >= 0.0) and np.all(o["var_data"] <= R * (1 + 1e-12))
        assert np.all(o["var_test"] >= 0.0) and np.all(o["var_test"] <= k0 * (1 + 1e-12))
    errs = (np.max(np.abs(a["mean_data"] - c["mean_data"])) / np.sqrt(k0),
            np.max(np.abs(a["var_data"] - c["var_data"])) / k0,
            np.max(np.abs(a["mean_test"] - c["mean_test"])) / np.sqrt(k0),
            np.max(np.abs(a["var_test"] - c["var_test"])) / k0)
    print("two plans", errs)
    assert max(errs) < 1e-9, errs


def test_long_100k_smoother(lib):
    """One series of 1e5 exposures with 1e4 test times: every smoothed moment
    at the data and at the test times against the oracle.

    At this size the oracle's own accuracy sets the tolerance.  Its smoother is
    the RTS recursion and the interpolation of Algorithm 1 as the paper prints
    them, in long double; both invert a predicted covariance, which is nearly
    singular where two exposures start almost together.  This series has three
    start pairs less than 0.01 s apart: just before them the oracle's smoothed
    variances err by up to 7.4e-7 of the prior variance, and elsewhere its
    test-time moments by up to 2.7e-9, measured against the dense posterior of
    301-exposure windows, to which the GPU agrees within 4e-16 (variances) and
    4e-14 (means) at the same points.  Exposures and test times within 0.1 day
    before a start pair closer than 0.02 s are held to 1e-5; elsewhere the data
    to 2e-9 and the test times to 1e-8."""
    b = W.long_100k()
    plan = lib.Plan(b.offsets, b.t_start, b.t_end, b.y, b.yerr)
    out = plan.smooth(b.sigma, b.omega0, b.quality, b.jitter, b.test_offsets, b.t_test, terms=True)
    out = {k: v.cpu().numpy() for k, v in out.items() if v is not None}
    s = b.series(0)
    L, mt, vt, md, vd, tm, tv = kalman.smooth(*_args(s), t_test=b.t_test, terms=True)
    k0 = float(np.sum(np.asarray(s["sigma"]) ** 2))
    ts = s["ts"]
    pairs = ts[1:][np.diff(ts) * 86400.0 < 0.02]
    near_d = np.zeros(len(ts), bool)
    near_t = np.zeros(len(b.t_test), bool)
    for tp in pairs:
        near_d |= (ts >= tp - 0.1) & (ts <= tp)
        near_t |= (b.t_test >= tp - 0.1) & (b.t_test <= tp)
    assert 0 < near_d.sum() < 200
    for near, tol_d, tol_t in ((False, 2e-9, 1e-8), (True, 1e-5, 1e-5)):
        d = near_d == near
        t = near_t == near
        errs_d = (np.max(np.abs(out["mean_data"] - md)[d], initial=0) / np.sqrt(k0),
                  np.max(np.abs(out["var_data"] - vd)[d], initial=0) / k0)
        errs_t = (np.max(np.abs(out["mean_test"] - mt)[t], initial=0) / np.sqrt(k0),
                  np.max(np.abs(out["var_test"] - vt)[t], initial=0) / k0,
                  np.max(np.abs(out["term_mean"] - tm)[t], initial=0) / np.sqrt(k0),
                  np.max(np.abs(out["term_var"] - tv)[t], initial=0) / k0)
        print(plan.stats(), "near" if near else "elsewhere", int(d.sum()), int(t.sum()), errs_d, errs_t)
        assert all(np.isfinite(errs_d)) and max(errs_d) < tol_d, (near, errs_d)
        assert all(np.isfinite(errs_t)) and max(errs_t) < tol_t, (near, errs_t)
    assert abs(out["loglik"][0] - L) < LL_TOL * abs(L)
    del plan
    _free()
