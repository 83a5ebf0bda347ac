"""GPU parity: the HIP library against the oracle on the same seeded inputs.

Tolerances: log-likelihood 1e-9 relative (|L_gpu - L_ref| / |L_ref|),
gradient 1e-6 (max_i |g_i - g_ref,i| / max(|g_ref,i|, 1e-3 max_j |g_ref,j|)).
"""
import math

import numpy as np
import pytest

import workloads as W
from oracle import dense, kalman

pytestmark = pytest.mark.gpu

LL_TOL = 1e-9
GRAD_TOL = 1e-6


def _oracle_ll(b):
    out = []
    for i in range(b.n_series):
        s = b.series(i)
        out.append(kalman.loglik(s["ts"], s["te"], s["y"], s["yerr"], s["sigma"], s["omega0"], s["quality"],
                                 s["jitter"]))
    return np.array(out)


def _plan(gp, b, **opt):
    return gp.Plan(b.offsets, b.t_start, b.t_end, b.y, b.yerr, **opt)


def _gpu_ll(gp, b, **opt):
    plan = _plan(gp, b, **opt)
    ll = plan.loglik(b.sigma, b.omega0, b.quality, b.jitter).cpu().numpy()
    return ll, plan


def _rel(a, b):
    return np.abs(a - b) / np.maximum(np.abs(b), 1e-300)


def _grad_err(g, ref):
    den = np.maximum(np.abs(ref), 1e-3 * np.max(np.abs(ref)))
    return np.max(np.abs(g - ref) / den)


@pytest.mark.parametrize("make", [W.small_single, W.small_multi])
def test_validation_scenarios_match_dense(lib, make):
    b = make()
    s = b.series(0)
    ref = dense.loglik(s["ts"], s["te"], s["y"], s["yerr"], s["sigma"], s["omega0"], s["quality"], s["jitter"])
    ll, _ = _gpu_ll(lib, b)
    print(make.__name__, ll[0], ref)
    assert _rel(ll[0], ref) < LL_TOL


def test_single_1k_matches_dense(lib):
    """The 1e3-exposure single series with its measurements drawn from the
    dense integrated GP itself (Cholesky of K + R, the oracle's covariance),
    as well as with the workload's surrogate signal."""
    b = W.single_1k()
    s = b.series(0)
    K = dense.covariance(s["ts"], s["te"], s["sigma"], s["omega0"], s["quality"])
    C = np.linalg.cholesky(K + np.diag(s["yerr"] ** 2))
    y_gp = C @ np.random.default_rng(1001).normal(size=len(s["ts"]))
    for y in (s["y"], y_gp):
        ref = dense.loglik(s["ts"], s["te"], y, s["yerr"], s["sigma"], s["omega0"], s["quality"], 0.0, K=K)
        plan = lib.Plan(b.offsets, b.t_start, b.t_end, y, b.yerr)
        ll = plan.loglik(b.sigma, b.omega0, b.quality, b.jitter).cpu().numpy()
        print("single_1k", ll[0], ref, plan.stats())
        assert _rel(ll[0], ref) < LL_TOL


@pytest.mark.parametrize("M,J", [(1, 1), (1, 2), (2, 2), (2, 3), (3, 3), (3, 4), (4, 2)])
def test_random_batches_match_oracle(lib, M, J):
    b = W.random_small_batch(100 * M + J, B=12, n_lo=1, n_hi=70, M=M, J=J)
    ref = _oracle_ll(b)
    ll, plan = _gpu_ll(lib, b, chunk_min=4, chunk_target=8)
    print(M, J, plan.stats(), np.max(_rel(ll, ref)))
    assert np.all(_rel(ll, ref) < LL_TOL)


@pytest.mark.parametrize("opt", [dict(single_chunk=1), dict(chunk_min=1, chunk_target=1), dict(chunk_min=4, chunk_target=6),
                                 dict(chunk_min=16, chunk_target=40), dict()])
def test_chunking_variants_agree(lib, opt):
    """Every chunking the planner can choose gives the same likelihood."""
    b = W.random_small_batch(7, B=9, n_lo=20, n_hi=120, M=2, J=3)
    ref = _oracle_ll(b)
    ll, plan = _gpu_ll(lib, b, **opt)
    print(opt, plan.stats(), np.max(_rel(ll, ref)))
    assert np.all(_rel(ll, ref) < LL_TOL)


def test_plain_filter_matches_batched(lib):
    b = W.random_small_batch(8, B=5, n_lo=10, n_hi=80, M=2, J=2)
    plan = _plan(lib, b, chunk_min=4, chunk_target=8)
    ll = plan.loglik(b.sigma, b.omega0, b.quality, b.jitter).cpu().numpy()
    lp = plan.plain_loglik(b.sigma, b.omega0, b.quality, b.jitter).cpu().numpy()
    ref = _oracle_ll(b)
    assert np.all(_rel(lp, ref) < LL_TOL)
    assert np.all(_rel(ll, lp) < LL_TOL)


def test_edge_cases(lib):
    """One exposure; all instantaneous; exact ties; zero jitter; a series of
    instantaneous points followed by exposures."""
    parts = [
        (np.array([1.0]), np.array([1.3]), np.array([0.2]), np.array([0.1])),
        (np.array([0.0, 0.1, 0.1, 0.5]), np.array([0.0, 0.1, 0.1, 0.5]), np.array([0.1, -0.2, 0.3, 0.0]),
         np.array([0.1, 0.2, 0.1, 0.3])),
        (np.array([0.0, 0.2, 0.2, 0.4]), np.array([0.2, 0.4, 0.3, 0.4]), np.array([0.3, 0.1, -0.1, 0.2]),
         np.full(4, 0.1)),
        (np.array([0.0, 0.05, 0.1, 0.15, 0.3]), np.array([0.0, 0.05, 0.2, 0.35, 0.3]),
         np.array([0.1, 0.2, 0.3, 0.1, 0.0]), np.full(5, 0.05)),
    ]
    off = np.concatenate([[0], np.cumsum([len(p[0]) for p in parts])])
    b = W.Batch(off.astype(np.int64), *[np.concatenate([p[i] for p in parts]) for i in range(4)],
                sigma=np.tile([[1.0, 0.3]], (4, 1)), omega0=np.tile([[3.0, 40.0]], (4, 1)),
                quality=np.tile([[0.7, 5.0]], (4, 1)), jitter=np.array([0.0, 0.05, 0.0, 0.02]))
    ref = _oracle_ll(b)
    for opt in (dict(), dict(chunk_min=1, chunk_target=1)):
        ll, _ = _gpu_ll(lib, b, **opt)
        assert np.all(_rel(ll, ref) < LL_TOL), (opt, ll, ref)


def test_parameter_regimes(lib):
    """Q below, at and above 1/2; very small and very large omega0 dt."""
    rng = np.random.default_rng(5)
    b = W.random_small_batch(21, B=6, n_lo=30, n_hi=60, M=2, J=2)
    b.quality[:] = np.array([[0.3, 0.5], [0.5 + 1e-9, 2.0], [0.45, 50.0], [0.5, 0.5], [1.0, 0.31], [30.0, 0.7]])
    b.omega0[:] = np.array([[1e-2, 3.0], [1e3, 5.0], [0.5, 2e3], [20.0, 0.1], [300.0, 1.0], [7.0, 50.0]])
    ref = _oracle_ll(b)
    ll, _ = _gpu_ll(lib, b, chunk_min=4, chunk_target=10)
    print(_rel(ll, ref))
    assert np.all(_rel(ll, ref) < LL_TOL)


def test_errors(lib):
    b = W.random_small_batch(3, B=2, n_lo=5, n_hi=10, M=1, J=1)
    plan = _plan(lib, b)
    bad = b.sigma.copy()
    bad[1, 0] = -1.0
    # hyperparameters are validated on the device: the plan forms report
    # through the per-series status, the one-shot forms by their return code
    with pytest.raises(lib.GpSsmError) as e:
        plan.loglik(bad, b.omega0, b.quality, b.jitter, check=True)
    assert e.value.code == -3
    with pytest.raises(lib.GpSsmError) as e:
        plan.loglik(b.sigma, b.omega0, b.quality, -np.ones(2), check=True)
    assert e.value.code == -3
    with pytest.raises(lib.GpSsmError) as e:
        lib.loglik(b.offsets, b.t_start, b.t_end, b.y, b.yerr, bad, b.omega0, b.quality, b.jitter)
    assert e.value.code == -3
    ts = b.t_start.copy()
    ts[[0, 1]] = ts[[1, 0]]
    with pytest.raises(lib.GpSsmError) as e:
        lib.Plan(b.offsets, ts, np.maximum(b.t_end, ts), b.y, b.yerr)
    assert e.value.code == -2
    # five mutually overlapping exposures
    with pytest.raises(lib.GpSsmError) as e:
        lib.Plan(np.array([0, 5]), np.arange(5) * 0.01, np.arange(5) * 0.01 + 1.0, np.zeros(5), np.ones(5))
    assert e.value.code == -4


@pytest.mark.parametrize("M,J,T", [(1, 1, 2.0), (2, 2, 2.0), (2, 3, 2.0), (3, 3, 2.0), (3, 4, 0.4), (4, 2, 2.0),
                                   (4, 4, 0.4)])
def test_gradient_matches_oracle(lib, M, J, T):
    """Each slot count's kernel (the batch reaches overlap depth J; with four
    the adjoint step keeps part of its state in LDS) against central
    differences of the oracle."""
    b = W.random_small_batch(300 + 10 * M + J, B=6, n_lo=5, n_hi=60, M=M, J=J, T=T)
    plan = _plan(lib, b, chunk_min=4, chunk_target=9)
    assert plan.stats()["max_slots"] == J
    ll, g = plan.loglik_grad(b.sigma, b.omega0, b.quality, b.jitter)
    ll = ll.cpu().numpy()
    g = g.cpu().numpy()
    ref = _oracle_ll(b)
    assert np.all(_rel(ll, ref) < LL_TOL)
    for i in range(b.n_series):
        s = b.series(i)
        gfd = kalman.loglik_grad_fd(s["ts"], s["te"], s["y"], s["yerr"], s["sigma"], s["omega0"], s["quality"],
                                    s["jitter"])
        err = _grad_err(g[i], gfd)
        print(i, err)
        assert err < GRAD_TOL, (i, g[i], gfd)


def test_gradient_matches_dense_analytic(lib):
    b = W.small_multi()
    b.jitter[:] = 0.04
    s = b.series(0)
    L, gref = dense.loglik_grad(s["ts"], s["te"], s["y"], s["yerr"], s["sigma"], s["omega0"], s["quality"], 0.04)
    for opt in (dict(), dict(chunk_min=2, chunk_target=3)):
        plan = _plan(lib, b, **opt)
        ll, g = plan.loglik_grad(b.sigma, b.omega0, b.quality, b.jitter)
        assert _rel(ll.cpu().numpy()[0], L) < LL_TOL
        assert _grad_err(g.cpu().numpy()[0], gref) < GRAD_TOL


def test_autograd_function(lib):
    import torch
    b = W.random_small_batch(31, B=3, n_lo=10, n_hi=30, M=2, J=2)
    plan = _plan(lib, b)
    s = torch.tensor(b.sigma, device="cuda", requires_grad=True)
    w = torch.tensor(b.omega0, device="cuda", requires_grad=True)
    q = torch.tensor(b.quality, device="cuda", requires_grad=True)
    j = torch.tensor(b.jitter, device="cuda", requires_grad=True)
    ll = lib.loglik_autograd(plan, s, w, q, j)
    wts = torch.tensor([1.0, -2.0, 0.5], dtype=torch.float64, device="cuda")
    (ll * wts).sum().backward()
    _, g = plan.loglik_grad(b.sigma, b.omega0, b.quality, b.jitter)
    g = g.cpu().numpy() * np.array([1.0, -2.0, 0.5])[:, None]
    assert np.allclose(s.grad.cpu().numpy(), g[:, 0:2], rtol=1e-14, atol=0)
    assert np.allclose(w.grad.cpu().numpy(), g[:, 2:4], rtol=1e-14, atol=0)
    assert np.allclose(q.grad.cpu().numpy(), g[:, 4:6], rtol=1e-14, atol=0)
    assert np.allclose(j.grad.cpu().numpy(), g[:, 6], rtol=1e-14, atol=0)


def test_long_series_multi_level_scan(lib):
    """One series split into thousands of chunks (more than 64 segments, so
    the scan over segment totals runs several segments per lane), plus a
    second short series: likelihood and gradient against the oracle."""
    b = W.random_small_batch(77, B=2, n_lo=6000, n_hi=6000, M=2, J=2, T=600.0)
    ref = _oracle_ll(b)
    for opt in (dict(chunk_min=1, chunk_target=1), dict(chunk_min=2, chunk_target=3), dict()):
        plan = _plan(lib, b, **opt)
        st = plan.stats()
        ll, g = plan.loglik_grad(b.sigma, b.omega0, b.quality, b.jitter)
        ll = ll.cpu().numpy()
        print(opt, st, _rel(ll, ref))
        assert np.all(_rel(ll, ref) < LL_TOL)
        if opt.get("chunk_target") == 1:
            assert st["n_segments"] > 64
            s = b.series(1)
            gfd = kalman.loglik_grad_fd(s["ts"], s["te"], s["y"], s["yerr"], s["sigma"], s["omega0"], s["quality"],
                                        s["jitter"])
            assert _grad_err(g.cpu().numpy()[1], gfd) < GRAD_TOL


def test_two_level_scan_with_several_totals_per_lane(lib):
    """A 300000-exposure single-instrument series cut at every quiet point:
    more than 4096 segments, so the second scan level runs over more than 64
    groups and each lane of the series-level scan walks several group
    totals.  Log-likelihood against the oracle; the gradient against that of
    the default chunking, whose scan has a different structure."""
    b = W.random_small_batch(91, B=1, n_lo=300000, n_hi=300000, M=1, J=1, T=30000.0)
    ref = _oracle_ll(b)
    plan = _plan(lib, b, chunk_min=1, chunk_target=1)
    st = plan.stats()
    assert st["n_segments"] > 64 * 64, st
    ll, g = plan.loglik_grad(b.sigma, b.omega0, b.quality, b.jitter)
    ll1 = plan.loglik(b.sigma, b.omega0, b.quality, b.jitter).cpu().numpy()
    ll, g = ll.cpu().numpy(), g.cpu().numpy()
    plan0 = _plan(lib, b)
    ll0, g0 = plan0.loglik_grad(b.sigma, b.omega0, b.quality, b.jitter)
    ll0, g0 = ll0.cpu().numpy(), g0.cpu().numpy()
    print(st, plan0.stats(), _rel(ll, ref), _rel(ll0, ref), _grad_err(g[0], g0[0]))
    assert np.all(_rel(ll, ref) < LL_TOL) and np.all(_rel(ll1, ref) < LL_TOL) and np.all(_rel(ll0, ref) < LL_TOL)
    assert _grad_err(g[0], g0[0]) < GRAD_TOL


def test_one_shot_entry_points(lib):
    """gp_ssm_loglik, gp_ssm_loglik_grad and gp_ssm_smooth (plan, run, destroy
    in one call) give the plan path's results bit for bit, and the oracle's."""
    b = W.random_small_batch(33, B=5, n_lo=3, n_hi=50, M=2, J=3)
    inputs = (b.offsets, b.t_start, b.t_end, b.y, b.yerr, b.sigma, b.omega0, b.quality, b.jitter)
    plan = _plan(lib, b)
    ll_p, g_p = plan.loglik_grad(b.sigma, b.omega0, b.quality, b.jitter)
    ll1 = lib.loglik(*inputs).cpu().numpy()
    ll2, g2 = lib.loglik_grad(*inputs)
    assert np.array_equal(ll1, ll_p.cpu().numpy()) and np.array_equal(ll2.cpu().numpy(), ll_p.cpu().numpy())
    assert np.array_equal(g2.cpu().numpy(), g_p.cpu().numpy())
    assert np.all(_rel(ll1, _oracle_ll(b)) < LL_TOL)
    tt = np.concatenate([np.linspace(b.series(i)["ts"].min() - 0.1, b.series(i)["te"].max() + 0.1, 9)
                         for i in range(b.n_series)])
    to = np.arange(b.n_series + 1, dtype=np.int64) * 9
    o1 = lib.smooth(*inputs, to, tt)
    o2 = plan.smooth(b.sigma, b.omega0, b.quality, b.jitter, to, tt)
    for k in ("mean_test", "var_test", "mean_data", "var_data"):
        assert np.array_equal(o1[k].cpu().numpy(), o2[k].cpu().numpy()), k
    assert np.all(o1["status"].cpu().numpy() == 0)
