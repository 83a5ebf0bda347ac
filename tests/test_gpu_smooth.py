"""GPU parity of the smoother: posterior of the exposure-averaged process at
the data and of the latent process at test times, against the oracle's
sequential RTS smoother with Algorithm 1 and against the dense posterior.

Tolerance: absolute 1e-9 times the prior scale (sum of sigma^2 for
variances, its square root for means)."""
import numpy as np
import pytest

import workloads as W
from oracle import dense, kalman

pytestmark = pytest.mark.gpu

TOL = 1e-9


def _run(lib, b, t_test, test_offsets, terms=False, **opt):
    plan = lib.Plan(b.offsets, b.t_start, b.t_end, b.y, b.yerr, **opt)
    out = plan.smooth(b.sigma, b.omega0, b.quality, b.jitter, test_offsets, t_test, terms=terms)
    return {k: (v.cpu().numpy() if v is not None else None) for k, v in out.items()}, plan


def _check(b, out, t_test, test_offsets, use_dense=False):
    for i in range(b.n_series):
        s = b.series(i)
        tt = t_test[test_offsets[i]:test_offsets[i + 1]]
        args = (s["ts"], s["te"], s["y"], s["yerr"], s["sigma"], s["omega0"], s["quality"], s["jitter"])
        L, mt, vt, md, vd = kalman.smooth(*args, t_test=tt)
        k0 = float(np.sum(np.asarray(s["sigma"]) ** 2))
        a, e = int(b.offsets[i]), int(b.offsets[i + 1])
        gm = out["mean_data"][a:e]
        gv = out["var_data"][a:e]
        tm = out["mean_test"][test_offsets[i]:test_offsets[i + 1]]
        tv = out["var_test"][test_offsets[i]:test_offsets[i + 1]]
        errs = (np.max(np.abs(gm - md), initial=0) / np.sqrt(k0), np.max(np.abs(gv - vd), initial=0) / k0,
                np.max(np.abs(tm - mt), initial=0) / np.sqrt(k0), np.max(np.abs(tv - vt), initial=0) / k0)
        print(i, errs)
        assert max(errs) < TOL, (i, errs)
        assert abs(out["loglik"][i] - L) < 1e-9 * abs(L)
        if use_dense:
            dmd, dvd, dmt, dvt = dense.posterior(*args, t_test=tt)
            assert np.max(np.abs(gm - dmd)) < 1e-9 * np.sqrt(k0)
            assert np.max(np.abs(gv - dvd)) < 1e-9 * k0
            assert np.max(np.abs(tm - dmt)) < 1e-9 * np.sqrt(k0)
            assert np.max(np.abs(tv - dvt)) < 1e-9 * k0


@pytest.mark.parametrize("make", [W.small_single, W.small_multi])
def test_validation_scenarios(lib, make):
    b = make()
    b.jitter[:] = 0.01
    for opt in (dict(), dict(chunk_min=2, chunk_target=3)):
        out, plan = _run(lib, b, b.t_test, b.test_offsets, **opt)
        _check(b, out, b.t_test, b.test_offsets, use_dense=True)


@pytest.mark.parametrize("opt", [dict(), dict(chunk_min=1, chunk_target=1), dict(chunk_min=5, chunk_target=7),
                                 dict(single_chunk=1)])
def test_random_batches(lib, opt):
    b = W.random_small_batch(41, B=7, n_lo=2, n_hi=50, M=2, J=3)
    rng = np.random.default_rng(3)
    parts = []
    for i in range(b.n_series):
        s = b.series(i)
        lo, hi = s["ts"].min(), s["te"].max()
        t = np.concatenate([rng.uniform(lo - 0.3, hi + 0.3, 23), s["ts"][:3], s["te"][-2:], [lo - 5.0, hi + 5.0]])
        parts.append(t)
    to = np.concatenate([[0], np.cumsum([len(p) for p in parts])]).astype(np.int64)
    tt = np.concatenate(parts)
    out, plan = _run(lib, b, tt, to, **opt)
    _check(b, out, tt, to)


def test_parameter_regimes(lib):
    b = W.random_small_batch(43, B=4, n_lo=20, n_hi=40, M=2, J=2)
    b.quality[:] = np.array([[0.3, 0.5], [0.5 + 1e-9, 2.0], [0.45, 50.0], [30.0, 0.7]])
    to = np.arange(b.n_series + 1, dtype=np.int64) * 15
    tt = np.concatenate([np.linspace(b.series(i)["ts"].min() - 0.1, b.series(i)["te"].max() + 0.1, 15)
                         for i in range(b.n_series)])
    out, plan = _run(lib, b, tt, to, chunk_min=3, chunk_target=5)
    _check(b, out, tt, to)


def test_long_series_many_segments(lib):
    """A 45000-exposure series with the mixed-cadence recipe of the 1e5-point
    smoothing workload (a fast Q=30 term beside a Q=1/sqrt(2) term): under
    default chunking, and with one-exposure chunks so that the scan over
    segment totals runs several segments per lane.  The series holds exposures
    that start within a second of each other, whose integrators are nearly
    equal: a backward sweep that inverts the predicted covariance loses
    accuracy there, and errors in the information form of the compositions
    show up here as non-finite or inaccurate smoothed moments."""
    b = W.long_100k(n=45000, n_test=4500, T=165.0)
    s = b.series(0)
    ref = kalman.smooth(s["ts"], s["te"], s["y"], s["yerr"], s["sigma"], s["omega0"], s["quality"], s["jitter"],
                        t_test=b.t_test, terms=True)
    k0 = float(np.sum(np.asarray(s["sigma"]) ** 2))
    for opt in (dict(), dict(chunk_min=1, chunk_target=1)):
        out, plan = _run(lib, b, b.t_test, b.test_offsets, terms=True, **opt)
        st = plan.stats()
        if opt:
            assert st["n_segments"] > 64
        L, mt, vt, md, vd, tm, tv = ref
        errs = (np.max(np.abs(out["mean_data"] - md)) / np.sqrt(k0), np.max(np.abs(out["var_data"] - vd)) / k0,
                np.max(np.abs(out["mean_test"] - mt)) / np.sqrt(k0), np.max(np.abs(out["var_test"] - vt)) / k0,
                np.max(np.abs(out["term_mean"] - tm)) / np.sqrt(k0), np.max(np.abs(out["term_var"] - tv)) / k0)
        print(opt, st["n_segments"], errs)
        assert all(np.isfinite(errs)) and max(errs) < TOL, (opt, errs)
        assert abs(out["loglik"][0] - L) < 1e-9 * abs(L)


@pytest.mark.parametrize("opt", [dict(), dict(chunk_min=1, chunk_target=1), dict(single_chunk=1)])
def test_component_posteriors(lib, opt):
    """Each term's own latent posterior at test times before, between, at and
    after the events (Appendix C, component-wise predictive means and
    variances) against the oracle, with the totals unchanged and equal to the
    row sums of the term means."""
    b = W.random_small_batch(47, B=5, n_lo=3, n_hi=60, M=3, J=3)
    rng = np.random.default_rng(11)
    parts = []
    for i in range(b.n_series):
        s = b.series(i)
        lo, hi = s["ts"].min(), s["te"].max()
        parts.append(np.concatenate([rng.uniform(lo - 0.3, hi + 0.3, 19), s["ts"][:2], s["te"][-2:],
                                     [lo - 4.0, hi + 4.0]]))
    to = np.concatenate([[0], np.cumsum([len(p) for p in parts])]).astype(np.int64)
    tt = np.concatenate(parts)
    out, plan = _run(lib, b, tt, to, terms=True, **opt)
    base, _ = _run(lib, b, tt, to, **opt)
    assert np.array_equal(out["mean_test"], base["mean_test"]) and np.array_equal(out["var_test"], base["var_test"])
    assert out["term_mean"].shape == (len(tt), 3)
    for i in range(b.n_series):
        s = b.series(i)
        sl = slice(int(to[i]), int(to[i + 1]))
        args = (s["ts"], s["te"], s["y"], s["yerr"], s["sigma"], s["omega0"], s["quality"], s["jitter"])
        L, mt, vt, md, vd, tm, tv = kalman.smooth(*args, t_test=tt[sl], terms=True)
        k0 = float(np.sum(np.asarray(s["sigma"]) ** 2))
        e = (np.max(np.abs(out["term_mean"][sl] - tm)) / np.sqrt(k0), np.max(np.abs(out["term_var"][sl] - tv)) / k0,
             np.max(np.abs(out["term_mean"][sl].sum(axis=1) - out["mean_test"][sl])) / np.sqrt(k0))
        print(i, e)
        assert max(e) < TOL, (i, e)


@pytest.mark.parametrize("M,J,T", [(3, 4, 0.4), (4, 2, 2.0), (4, 4, 0.4)])
def test_four_slots_and_four_terms(lib, M, J, T):
    """The smoother's kernels for four overlapping exposures and for four terms
    (dense batches reach the overlap depth they name), total and per-term
    posteriors against the oracle."""
    b = W.random_small_batch(70 + 10 * M + J, B=4, n_lo=10, n_hi=50, M=M, J=J, T=T)
    rng = np.random.default_rng(17)
    parts = []
    for i in range(b.n_series):
        s = b.series(i)
        lo, hi = s["ts"].min(), s["te"].max()
        parts.append(np.concatenate([rng.uniform(lo - 0.05, hi + 0.05, 15), s["te"][:2]]))
    to = np.concatenate([[0], np.cumsum([len(p) for p in parts])]).astype(np.int64)
    tt = np.concatenate(parts)
    out, plan = _run(lib, b, tt, to, terms=True, chunk_min=3, chunk_target=5)
    assert plan.stats()["max_slots"] == J
    _check(b, out, tt, to)
    for i in range(b.n_series):
        s = b.series(i)
        sl = slice(int(to[i]), int(to[i + 1]))
        *_, tm, tv = kalman.smooth(s["ts"], s["te"], s["y"], s["yerr"], s["sigma"], s["omega0"], s["quality"],
                                   s["jitter"], t_test=tt[sl], terms=True)
        k0 = float(np.sum(np.asarray(s["sigma"]) ** 2))
        assert np.max(np.abs(out["term_mean"][sl] - tm)) < TOL * np.sqrt(k0)
        assert np.max(np.abs(out["term_var"][sl] - tv)) < TOL * k0


def test_scan_equals_sequential(lib):
    """The time-parallel scan against the same computation without time
    splitting (one chunk per series, so one lane runs each series from its
    prior): log-likelihood within 1e-12 relative, and the one-lane plain
    filter; smoothed moments within 1e-12 of the prior standard deviation /
    variance."""
    b = W.random_small_batch(808, B=6, n_lo=60, n_hi=300, M=2, J=3, T=8.0)
    nt = 25
    tt = np.concatenate([np.linspace(b.series(i)["ts"].min() - 0.1, b.series(i)["te"].max() + 0.1, nt)
                         for i in range(b.n_series)])
    to = np.arange(b.n_series + 1, dtype=np.int64) * nt
    k0 = np.sum(np.asarray(b.sigma) ** 2, axis=1)
    res = {}
    for name, opt in (("seq", dict(single_chunk=1)), ("scan", dict(chunk_min=1, chunk_target=2)), ("dflt", dict())):
        plan = lib.Plan(b.offsets, b.t_start, b.t_end, b.y, b.yerr, **opt)
        o = plan.smooth(b.sigma, b.omega0, b.quality, b.jitter, to, tt)
        res[name] = {k: v.cpu().numpy() for k, v in o.items() if v is not None}
        res[name]["plain"] = plan.plain_loglik(b.sigma, b.omega0, b.quality, b.jitter).cpu().numpy()
        print(name, plan.stats())
    seq = res["seq"]
    for name in ("scan", "dflt"):
        r = res[name]
        assert np.max(np.abs(r["loglik"] - seq["loglik"]) / np.abs(seq["loglik"])) < 1e-12
        assert np.max(np.abs(r["loglik"] - seq["plain"]) / np.abs(seq["plain"])) < 1e-12
        for i in range(b.n_series):
            lo, hi = int(b.offsets[i]), int(b.offsets[i + 1])
            s0, s1 = int(to[i]), int(to[i + 1])
            e = (np.max(np.abs(r["mean_data"][lo:hi] - seq["mean_data"][lo:hi])) / np.sqrt(k0[i]),
                 np.max(np.abs(r["var_data"][lo:hi] - seq["var_data"][lo:hi])) / k0[i],
                 np.max(np.abs(r["mean_test"][s0:s1] - seq["mean_test"][s0:s1])) / np.sqrt(k0[i]),
                 np.max(np.abs(r["var_test"][s0:s1] - seq["var_test"][s0:s1])) / k0[i])
            print(name, i, e)
            assert max(e) < 1e-12, (name, i, e)
