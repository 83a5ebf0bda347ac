"""GPU parity against stored oracle values (tests/golden/, each written by the
committed script beside it, which calls only workloads and oracle/):

* two series whose scan, cut at every quiet point, runs its second level:
  32000 exposures from the generator of the 1e7-exposure workload (three
  terms, up to four overlapping exposures, scan width 6) and a four-term
  series (width 8); log-likelihood and gradient against the sequential
  long-double oracle and its central differences;
* the 1024-series gradient batch: the first 500 exposures of eight series
  against the dense oracle's analytic gradient (quadrature + Cholesky);
* the smoother where two exposures start almost together, against the dense
  posterior: the 60-exposure case with a 3 ms start pair and 301-exposure
  windows of the 1e5-exposure workload around its four start pairs closer
  than 0.02 s.

Tolerances: log-likelihood 1e-9 relative, gradient 1e-6 (relative to
max(|g_i|, 1e-3 max|g|)), smoothed means 1e-9 of the prior standard
deviation and variances 1e-9 of the prior variance.
"""
import json
import os

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
GOLD = os.path.join(HERE, "golden")
LL_TOL = 1e-9
GRAD_TOL = 1e-6
POST_TOL = 1e-9


def _load(name):
    with open(os.path.join(GOLD, name)) as fh:
        return json.load(fh)


def _grad_err(g, ref):
    ref = np.asarray(ref)
    den = np.maximum(np.abs(ref), 1e-3 * np.max(np.abs(ref)))
    return np.max(np.abs(np.asarray(g) - ref) / den)


@pytest.mark.parametrize("case", ["c5_prefix", "m4"])
def test_long_scan_two_levels_against_oracle(lib, case):
    rows = {r["name"]: r for r in _load("kalman_long_scan.json")["cases"]}
    r = rows[case]
    b = getattr(W, r["generator"])(**r["kwargs"])
    for opt in (dict(chunk_min=1, chunk_target=1), dict()):
        plan = lib.Plan(b.offsets, b.t_start, b.t_end, b.y, b.yerr, **opt)
        st = plan.stats()
        ll, g = plan.loglik_grad(b.sigma, b.omega0, b.quality, b.jitter)
        ll, g = float(ll.cpu().numpy()[0]), g.cpu().numpy()[0]
        rel = abs(ll - r["loglik"]) / abs(r["loglik"])
        gref = np.asarray(r["grad_fd"])
        if b.jitter[0] == 0.0:
            # the likelihood depends on the jitter through its square: the
            # derivative at zero is exactly 0, where the difference quotient,
            # one sided at the boundary, is not
            assert g[-1] == 0.0
            g, gref = g[:-1], gref[:-1]
        ge = _grad_err(g, gref)
        print(case, opt, st, rel, ge)
        if opt:
            assert st["n_segments"] > 64, st
        if case == "c5_prefix":
            assert st["max_slots"] == 4 and b.n_terms == 3
        else:
            assert b.n_terms == 4
        assert rel < LL_TOL
        assert ge < GRAD_TOL


def test_grad_1024_dense_subsets(lib):
    gold = _load("dense_grad_1024.json")["rows"]
    full = W.grad_1024()
    parts = []
    for r in gold:
        s = full.series(r["series"])
        n = r["n"]
        parts.append((s["ts"][:n], s["te"][:n], s["y"][:n], s["yerr"][:n]))
    idx = [r["series"] for r in gold]
    off = np.concatenate([[0], np.cumsum([len(p[0]) for p in parts])]).astype(np.int64)
    cat = [np.concatenate([p[k] for p in parts]) for k in range(4)]
    plan = lib.Plan(off, *cat)
    ll, g = plan.loglik_grad(full.sigma[idx], full.omega0[idx], full.quality[idx], full.jitter[idx])
    ll, g = ll.cpu().numpy(), g.cpu().numpy()
    for k, r in enumerate(gold):
        rel = abs(ll[k] - r["loglik"]) / abs(r["loglik"])
        ge = _grad_err(g[k], r["grad"])
        print("series", r["series"], rel, ge)
        assert rel < LL_TOL
        assert ge < GRAD_TOL


def test_smoother_near_coincident_starts_dense(lib):
    cases = _load("dense_smoother_pairs.json")["cases"]
    assert [c["name"] for c in cases] == ["pair3ms"] + [f"long_100k_w{k}" for k in range(4)]
    for c in cases:
        ts, te, y, yerr = (np.asarray(c[k]) for k in ("ts", "te", "y", "yerr"))
        tt = np.asarray(c["t_test"])
        sig = np.asarray(c["sigma"])[None, :]
        w0 = np.asarray(c["omega0"])[None, :]
        q = np.asarray(c["quality"])[None, :]
        jit = np.array([c["jitter"]])
        k0 = float(np.sum(sig ** 2))
        assert np.min(np.diff(ts)) * 86400.0 < 0.02
        for opt in (dict(), dict(chunk_min=1, chunk_target=1)):
            plan = lib.Plan(np.array([0, len(ts)], dtype=np.int64), ts, te, y, yerr, **opt)
            o = plan.smooth(sig, w0, q, jit, np.array([0, len(tt)], dtype=np.int64), tt)
            md, vd, mt, vt = (o[k].cpu().numpy() for k in ("mean_data", "var_data", "mean_test", "var_test"))
            errs = (np.max(np.abs(md - c["mean_data"])) / np.sqrt(k0), np.max(np.abs(vd - c["var_data"])) / k0,
                    np.max(np.abs(mt - c["mean_test"])) / np.sqrt(k0), np.max(np.abs(vt - c["var_test"])) / k0)
            print(c["name"], opt, errs)
            assert max(errs) < POST_TOL, (c["name"], opt, errs)
