"""GPU parity for terms other than the SHO: the real exponential term
sigma^2 exp(-omega0 |tau|) (the celerite term of Appendix A with b = d = 0,
set by gp_ssm_plan_set_term_kinds), alone and mixed with SHO terms, against
the oracle (log-likelihood, central-difference gradient, smoother); and the
Matern-3/2 kernel through the SHO term at Q = 1/2 against the dense GP with
that kernel written out.

Tolerances as in test_gpu_parity: log-likelihood 1e-9 relative, gradient
1e-6 (relative to max(|g_i|, 1e-3 max|g|)), smoothed moments 1e-9 of the
prior standard deviation / variance."""
import math

import numpy as np
import pytest
from scipy.linalg import cho_factor, cho_solve

import workloads as W
from oracle import dense, kalman

pytestmark = pytest.mark.gpu

KIND_SETS = [["real"], ["real", "sho"], ["sho", "real", "real"], ["real", "real", "sho", "sho"]]


def _args(s):
    return (s["ts"], s["te"], s["y"], s["yerr"], s["sigma"], s["omega0"], s["quality"], s["jitter"])


def _grad_err(g, ref):
    den = np.maximum(np.abs(ref), 1e-3 * np.max(np.abs(ref)))
    return np.max(np.abs(g - ref) / den)


def _batch(kinds, seed):
    M = len(kinds)
    b = W.random_small_batch(seed, B=5, n_lo=10, n_hi=80, M=M, J=3)
    for m, k in enumerate(kinds):
        if k == "real":
            b.quality[:, m] = -1.0  # not read for a real term
    return b


@pytest.mark.parametrize("kinds", KIND_SETS)
def test_real_terms_match_oracle(lib, kinds):
    M = len(kinds)
    b = _batch(kinds, 500 + M)
    ref = np.array([kalman.loglik(*_args(b.series(i)), kinds=kinds) for i in range(b.n_series)])
    for opt in (dict(chunk_min=1, chunk_target=1), dict(chunk_min=4, chunk_target=9), dict()):
        plan = lib.Plan(b.offsets, b.t_start, b.t_end, b.y, b.yerr, **opt)
        plan.set_term_kinds(kinds)
        ll, g, st = plan.loglik_grad(b.sigma, b.omega0, b.quality, b.jitter, status=True)
        ll, g, st = ll.cpu().numpy(), g.cpu().numpy(), st.cpu().numpy()
        assert np.all(st == 0)
        rel = np.abs(ll - ref) / np.abs(ref)
        print(kinds, opt, plan.stats()["max_slots"], rel.max())
        assert np.all(rel < 1e-9)
        l1 = plan.loglik(b.sigma, b.omega0, b.quality, b.jitter).cpu().numpy()
        assert np.all(np.abs(l1 - ref) < 1e-9 * np.abs(ref))
    for i in (0, 3):
        s = b.series(i)
        gfd = kalman.loglik_grad_fd(*_args(s), kinds=kinds)
        real_q = [2 * M + m for m, k in enumerate(kinds) if k == "real"]
        assert np.all(g[i][real_q] == 0.0)
        e = _grad_err(g[i], gfd)
        print("gradient", i, e)
        assert e < 1e-6, (i, g[i], gfd)


def test_real_term_smoother_matches_oracle(lib):
    kinds = ["sho", "real"]
    b = _batch(kinds, 601)
    tt = np.concatenate([np.linspace(b.series(i)["ts"].min() - 0.05, b.series(i)["te"].max() + 0.05, 13)
                         for i in range(b.n_series)])
    to = np.arange(b.n_series + 1, dtype=np.int64) * 13
    plan = lib.Plan(b.offsets, b.t_start, b.t_end, b.y, b.yerr, chunk_min=4, chunk_target=8)
    plan.set_term_kinds(kinds)
    o = plan.smooth(b.sigma, b.omega0, b.quality, b.jitter, to, tt, terms=True)
    o = {k: v.cpu().numpy() for k, v in o.items() if v is not None}
    for i in range(b.n_series):
        s = b.series(i)
        L, mt, vt, md, vd, tm, tv = kalman.smooth(*_args(s), t_test=tt[to[i]:to[i + 1]], terms=True, kinds=kinds)
        k0 = float(np.sum(np.asarray(s["sigma"]) ** 2))
        a, e = int(b.offsets[i]), int(b.offsets[i + 1])
        errs = (np.max(np.abs(o["mean_data"][a:e] - md)) / math.sqrt(k0), np.max(np.abs(o["var_data"][a:e] - vd)) / k0,
                np.max(np.abs(o["mean_test"][to[i]:to[i + 1]] - mt)) / math.sqrt(k0),
                np.max(np.abs(o["var_test"][to[i]:to[i + 1]] - vt)) / k0,
                np.max(np.abs(o["term_mean"][to[i]:to[i + 1]] - tm)) / math.sqrt(k0),
                np.max(np.abs(o["term_var"][to[i]:to[i + 1]] - tv)) / k0)
        print(i, errs)
        assert max(errs) < 1e-9
        assert abs(o["loglik"][i] - L) < 1e-9 * abs(L)


def test_matern32_through_sho_at_half_against_dense(lib):
    """A Matern-3/2 term (sigma, rho) passed as the SHO term (sigma,
    sqrt3/rho, 1/2), against the dense GP whose kernel is the Matern-3/2
    kernel written out (same quadrature as the dense oracle)."""
    b = W.random_small_batch(602, B=1, n_lo=40, n_hi=40, M=1, J=2)
    s = b.series(0)
    sig, rho = 0.8, 0.09
    r3 = math.sqrt(3.0) / rho

    def matern(u):
        a = r3 * np.abs(u)
        return sig * sig * (1 + a) * np.exp(-a)

    ts, te = s["ts"], s["te"]
    K = dense._pair_block(ts[:, None], te[:, None], ts[None, :], te[None, :], matern, r3)
    Ky = 0.5 * (K + K.T) + np.diag(s["yerr"] ** 2 + s["jitter"] ** 2)
    cf = cho_factor(Ky, lower=True)
    y = s["y"]
    ref = float(-0.5 * y @ cho_solve(cf, y) - np.sum(np.log(np.diag(cf[0]))) - 0.5 * len(y) * math.log(2 * math.pi))
    plan = lib.Plan(b.offsets, b.t_start, b.t_end, b.y, b.yerr)
    ll = plan.loglik([[sig]], [[r3]], [[0.5]], b.jitter).cpu().numpy()
    print(ll[0], ref)
    assert abs(ll[0] - ref) < 1e-9 * abs(ref)


def test_term_kinds_must_match_the_call(lib):
    b = _batch(["real", "sho"], 603)
    plan = lib.Plan(b.offsets, b.t_start, b.t_end, b.y, b.yerr)
    plan.set_term_kinds(["real", "sho"])
    with pytest.raises(lib.GpSsmError) as e:
        plan.loglik(np.ones((5, 3)), np.ones((5, 3)), np.ones((5, 3)), b.jitter)
    assert e.value.code == -1
    plan.set_term_kinds(None)
    ll, st = plan.loglik(b.sigma, b.omega0, np.ones_like(b.quality), b.jitter, status=True)
    assert np.all(st.cpu().numpy() == 0)
