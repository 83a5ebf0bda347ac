"""GPU tests of the boundary's contract (include/gp_ssm.h): per-series status
and NaN outputs, empty series, hyperparameters in host memory, graph replay,
the batching pin and bitwise determinism.

Tolerances as in test_gpu_parity (log-likelihood 1e-9 relative, gradient
1e-6); where two runs of the library must agree, they must agree bit for bit
or to 1e-13 where the text says so.
"""
import ctypes

import numpy as np
import pytest

import workloads as W
from oracle import kalman

pytestmark = pytest.mark.gpu

LL_TOL = 1e-9
GRAD_TOL = 1e-6
EPARAM, ENUMERIC = -3, -5


def _oracle_ll(b):
    out = []
    for i in range(b.n_series):
        s = b.series(i)
        out.append(kalman.loglik(s["ts"], s["te"], s["y"], s["yerr"], s["sigma"], s["omega0"], s["quality"],
                                 s["jitter"]))
    return np.array(out)


def _rel(a, b):
    return np.abs(a - b) / np.maximum(np.abs(b), 1e-300)


def _grad_err(g, ref):
    den = np.maximum(np.abs(ref), 1e-3 * np.max(np.abs(ref)))
    return np.max(np.abs(g - ref) / den)


def _np(*ts):
    return [t.cpu().numpy() for t in ts]


def _inputs(b):
    return (b.offsets, b.t_start, b.t_end, b.y, b.yerr, b.sigma, b.omega0, b.quality, b.jitter)


def test_invalid_hyperparameters_isolated(lib):
    """A series with a negative sigma (or a negative jitter) gets status
    GP_SSM_EPARAM and NaN outputs from the plan forms, which return 0; the
    other series are bit-identical to a run in which that series is valid.
    The one-shot forms return GP_SSM_EPARAM."""
    b = W.random_small_batch(41, B=4, n_lo=10, n_hi=40, M=2, J=2)
    plan = lib.Plan(b.offsets, b.t_start, b.t_end, b.y, b.yerr, chunk_min=4, chunk_target=8)
    ll0, g0, st0 = _np(*plan.loglik_grad(b.sigma, b.omega0, b.quality, b.jitter, status=True))
    assert np.all(st0 == 0)
    for what in ("sigma", "jitter"):
        sig, jit = b.sigma.copy(), b.jitter.copy()
        if what == "sigma":
            sig[1, 0] = -1.0
        else:
            jit[1] = -0.1
        ll, g, st = _np(*plan.loglik_grad(sig, b.omega0, b.quality, jit, status=True))
        assert list(st) == [0, EPARAM, 0, 0], (what, st)
        assert np.isnan(ll[1]) and np.all(np.isnan(g[1]))
        keep = [0, 2, 3]
        assert np.array_equal(ll[keep], ll0[keep]) and np.array_equal(g[keep], g0[keep])
        l1, s1 = _np(*plan.loglik(sig, b.omega0, b.quality, jit, status=True))
        assert list(s1) == [0, EPARAM, 0, 0] and np.isnan(l1[1]) and np.array_equal(l1[keep], ll0[keep])
        with pytest.raises(lib.GpSsmError) as e:
            plan.loglik(sig, b.omega0, b.quality, jit, check=True)
        assert e.value.code == EPARAM
        with pytest.raises(lib.GpSsmError) as e:
            lib.loglik_grad(b.offsets, b.t_start, b.t_end, b.y, b.yerr, sig, b.omega0, b.quality, jit)
        assert e.value.code == EPARAM
        # the smoother: NaN for that series, the others unchanged
        tt = np.concatenate([np.linspace(b.series(i)["ts"].min(), b.series(i)["te"].max(), 5)
                             for i in range(b.n_series)])
        to = np.arange(b.n_series + 1, dtype=np.int64) * 5
        o_bad = plan.smooth(sig, b.omega0, b.quality, jit, to, tt)
        o_ok = plan.smooth(b.sigma, b.omega0, b.quality, b.jitter, to, tt)
        assert list(o_bad["status"].cpu().numpy()) == [0, EPARAM, 0, 0]
        mt_bad, mt_ok = o_bad["mean_test"].cpu().numpy(), o_ok["mean_test"].cpu().numpy()
        assert np.all(np.isnan(mt_bad[5:10])) and np.array_equal(mt_bad[:5], mt_ok[:5])
        md_bad = o_bad["mean_data"].cpu().numpy()
        n1 = slice(int(b.offsets[1]), int(b.offsets[2]))
        assert np.all(np.isnan(md_bad[n1]))


def test_numeric_failure_isolated(lib):
    """sigma = 1e200 passes validation but its square overflows: that series
    gets status GP_SSM_ENUMERIC and NaN log-likelihood and gradient, the other
    four are bit-identical to a clean run of the same plan, and the one-shot
    forms return GP_SSM_ENUMERIC."""
    b = W.random_small_batch(42, B=5, n_lo=10, n_hi=50, M=2, J=3)
    plan = lib.Plan(b.offsets, b.t_start, b.t_end, b.y, b.yerr)
    ll0, g0, st0 = _np(*plan.loglik_grad(b.sigma, b.omega0, b.quality, b.jitter, status=True))
    sig = b.sigma.copy()
    sig[2, 1] = 1e200
    ll, g, st = _np(*plan.loglik_grad(sig, b.omega0, b.quality, b.jitter, status=True))
    print(st, ll)
    assert list(st) == [0, 0, ENUMERIC, 0, 0]
    assert np.isnan(ll[2]) and np.all(np.isnan(g[2]))
    keep = [0, 1, 3, 4]
    assert np.array_equal(ll[keep], ll0[keep]) and np.array_equal(g[keep], g0[keep])
    assert np.all(_rel(ll0, _oracle_ll(b)) < LL_TOL)
    with pytest.raises(lib.GpSsmError) as e:
        lib.loglik(b.offsets, b.t_start, b.t_end, b.y, b.yerr, sig, b.omega0, b.quality, b.jitter)
    assert e.value.code == ENUMERIC


def test_empty_series(lib):
    """Series without measurements between and after others: log-likelihood
    0, gradient 0, status 0, the prior at their test times; the others match
    the oracle.  A batch of empty series alone gives zeros too."""
    import torch
    b = W.random_small_batch(43, B=3, n_lo=15, n_hi=40, M=2, J=2)
    parts = [b.series(0), None, b.series(1), b.series(2), None]
    idx = [0, None, 1, 2, None]
    lens = [0 if p is None else len(p["ts"]) for p in parts]
    off = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    cat = lambda k: np.concatenate([p[k] for p in parts if p is not None])
    pick = lambda a: np.stack([a[i] if i is not None else a[0] for i in idx])
    e = W.Batch(off, cat("ts"), cat("te"), cat("y"), cat("yerr"), pick(b.sigma), pick(b.omega0), pick(b.quality),
                np.array([b.jitter[i] if i is not None else 0.0 for i in idx]))
    ref = _oracle_ll(b)
    for opt in (dict(), dict(chunk_min=1, chunk_target=1)):
        plan = lib.Plan(e.offsets, e.t_start, e.t_end, e.y, e.yerr, **opt)
        ll, g, st = _np(*plan.loglik_grad(e.sigma, e.omega0, e.quality, e.jitter, status=True))
        assert np.all(st == 0)
        assert ll[1] == 0.0 and ll[4] == 0.0 and np.all(g[[1, 4]] == 0.0)
        assert np.all(_rel(ll[[0, 2, 3]], ref) < LL_TOL)
        tt = np.array([0.3, 0.7, 0.1, 0.5, 0.9, 0.2, 0.4])
        to = np.array([0, 2, 4, 5, 6, 7], dtype=np.int64)
        o = plan.smooth(e.sigma, e.omega0, e.quality, e.jitter, to, tt, terms=True)
        mt, vt, tv = _np(o["mean_test"], o["var_test"], o["term_var"])
        for i in (2, 3, 6):  # test times of the empty series 1 and 4
            ser = 1 if i < 4 else 4
            assert mt[i] == 0.0 and vt[i] == pytest.approx(np.sum(e.sigma[ser] ** 2), rel=1e-15)
            assert np.allclose(tv[i], e.sigma[ser] ** 2, rtol=1e-15)
    z = np.zeros(0)
    plan = lib.Plan(np.array([0, 0, 0], dtype=np.int64), z, z, z, z)
    ll, g = _np(*plan.loglik_grad(np.ones((2, 1)), np.ones((2, 1)), np.ones((2, 1)), np.zeros(2)))
    assert np.all(ll == 0.0) and np.all(g == 0.0)
    del torch


def test_host_hyperparameters(lib):
    """Hyperparameters passed as host arrays (copied on the stream) give the
    same results as device arrays; output arrays in host memory are refused."""
    import torch
    b = W.random_small_batch(44, B=3, n_lo=10, n_hi=30, M=2, J=2)
    plan = lib.Plan(b.offsets, b.t_start, b.t_end, b.y, b.yerr)
    ll_d, g_d = _np(*plan.loglik_grad(b.sigma, b.omega0, b.quality, b.jitter))
    L = lib.library()
    ll = torch.empty(3, dtype=torch.float64, device="cuda")
    g = torch.empty(3, 7, dtype=torch.float64, device="cuda")
    hs = [np.ascontiguousarray(a, dtype=np.float64) for a in (b.sigma, b.omega0, b.quality, b.jitter)]
    hp = [ctypes.c_void_p(a.ctypes.data) for a in hs]
    rc = L.gp_ssm_plan_loglik_grad(plan._h, 2, *hp, ctypes.c_void_p(ll.data_ptr()), ctypes.c_void_p(g.data_ptr()),
                                   None, lib._stream())
    assert rc == 0
    assert np.array_equal(ll.cpu().numpy(), ll_d) and np.array_equal(g.cpu().numpy(), g_d)
    host_out = np.zeros(3)
    rc = L.gp_ssm_plan_loglik(plan._h, 2, *hp, ctypes.c_void_p(host_out.ctypes.data), None, lib._stream())
    assert rc == -1


def test_graph_replays_match_direct_launches(lib):
    """The captured step, replayed with other hyperparameters and other output
    buffers and with eager work and synchronisations between replays, gives
    the results of launching the same kernels one by one (kernel timing on
    switches the replay off), bit for bit, on every replay."""
    import torch
    b = W.random_small_batch(45, B=7, n_lo=20, n_hi=200, M=3, J=3)
    plan = lib.Plan(b.offsets, b.t_start, b.t_end, b.y, b.yerr, chunk_min=4, chunk_target=12)
    rng = np.random.default_rng(0)
    thetas = [(b.sigma * f, b.omega0 * h, b.quality, b.jitter) for f, h in
              ((1.0, 1.0), (1.3, 0.7), (0.8, 1.9), (1.0, 1.0), (1.1, 1.05))]
    direct = []
    lib.profile_enable(True)
    try:
        for th in thetas:
            direct.append(_np(*plan.loglik_grad(*th)) + _np(plan.loglik(*th)))
    finally:
        lib.profile_enable(False)
    for rep in range(2):
        for k, th in enumerate(thetas):
            junk = torch.randn(1000, device="cuda").sum()  # eager work between replays
            ll, g = plan.loglik_grad(*th)
            l1 = plan.loglik(*th)
            torch.cuda.synchronize()
            got = _np(ll, g, l1)
            for a, d in zip(got, direct[k]):
                assert np.array_equal(a, d), (rep, k)
            del junk
    assert np.all(_rel(direct[0][0], _oracle_ll(b)) < LL_TOL)
    del rng


def test_batching_pin(lib):
    """Each series of a batch gives its own one-series result: with the same
    chunk length the per-series work is the same, so log-likelihood and
    gradient agree to 1e-13 (bit for bit in practice)."""
    b = W.random_small_batch(46, B=6, n_lo=30, n_hi=400, M=2, J=3, T=40.0)
    plan = lib.Plan(b.offsets, b.t_start, b.t_end, b.y, b.yerr, chunk_min=8, chunk_target=16)
    ll, g = _np(*plan.loglik_grad(b.sigma, b.omega0, b.quality, b.jitter))
    nbit = 0
    for i in range(b.n_series):
        s = b.subset([i])
        p1 = lib.Plan(s.offsets, s.t_start, s.t_end, s.y, s.yerr, chunk_min=8, chunk_target=16)
        l1, g1 = _np(*p1.loglik_grad(s.sigma, s.omega0, s.quality, s.jitter))
        print(i, l1[0], ll[i], _grad_err(g1[0], g[i]))
        assert _rel(l1[0], ll[i]) < 1e-13 and _grad_err(g1[0], g[i]) < 1e-13
        nbit += int(l1[0] == ll[i] and np.array_equal(g1[0], g[i]))
    print("bitwise equal series:", nbit, "of", b.n_series)


def test_bitwise_determinism(lib):
    """Two runs of a batch (hundreds of work waves, launched in an order with
    ties) give the same bits."""
    b = W.random_small_batch(47, B=40, n_lo=200, n_hi=3000, M=3, J=3, T=30.0)
    plan = lib.Plan(b.offsets, b.t_start, b.t_end, b.y, b.yerr, chunk_min=4, chunk_target=6)
    r1 = _np(*plan.loglik_grad(b.sigma, b.omega0, b.quality, b.jitter))
    plan2 = lib.Plan(b.offsets, b.t_start, b.t_end, b.y, b.yerr, chunk_min=4, chunk_target=6)
    r2 = _np(*plan2.loglik_grad(b.sigma, b.omega0, b.quality, b.jitter))
    r3 = _np(*plan.loglik_grad(b.sigma, b.omega0, b.quality, b.jitter))
    print(plan.stats())
    assert plan.stats()["n_chunks"] > 64 * 4
    for a, c, d in zip(r1, r2, r3):
        assert np.array_equal(a, c) and np.array_equal(a, d)


def test_record_rounds_match_whole_layout(lib):
    """With a record budget too small for the whole event layout, the gradient
    and the smoother run in rounds of work waves over a reused slot buffer
    (3000 series, more work waves than the GPU holds workgroups at once, so
    several rounds); results equal those of the default layout bit for bit,
    and the record buffer is the bounded one."""
    b = W.random_small_batch(48, B=3000, n_lo=10, n_hi=40, M=3, J=3, T=4.0)
    p0 = lib.Plan(b.offsets, b.t_start, b.t_end, b.y, b.yerr)
    p1 = lib.Plan(b.offsets, b.t_start, b.t_end, b.y, b.yerr, record_budget=1)
    r0 = _np(*p0.loglik_grad(b.sigma, b.omega0, b.quality, b.jitter))
    r1 = _np(*p1.loglik_grad(b.sigma, b.omega0, b.quality, b.jitter))
    s0, s1 = p0.stats(), p1.stats()
    D = 2 * 3 + s0["max_slots"]
    whole = 8 * (D + D * (D + 1) // 2) * s0["n_events_padded"]
    print(s0, s1, whole)
    assert s0["record_bytes"] == whole and s1["record_bytes"] < whole
    for a, c in zip(r0, r1):
        assert np.array_equal(a, c)
    tt = np.concatenate([np.linspace(0.0, 4.0, 3) for _ in range(b.n_series)])
    to = np.arange(b.n_series + 1, dtype=np.int64) * 3
    o0 = p0.smooth(b.sigma, b.omega0, b.quality, b.jitter, to, tt)
    o1 = p1.smooth(b.sigma, b.omega0, b.quality, b.jitter, to, tt)
    for k in ("mean_test", "var_test", "mean_data", "var_data"):
        assert np.array_equal(o0[k].cpu().numpy(), o1[k].cpu().numpy()), k
    assert np.all(_rel(r0[0][:5], _oracle_ll(b.subset(range(5)))) < LL_TOL)
