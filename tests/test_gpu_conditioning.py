"""GPU parity on nearly noise-free, densely sampled series (measurement
errors 1e-5 ... 1e-9 of the signal, many samples per correlation time),
against the high-precision dense oracle (mpmath, closed-form exposure
integrals): log-likelihood at 1e-9 relative and gradient at 1e-6, with the
default chunking, one chunk per series, and chunks of 4-8 events.

Here each measurement is almost predicted by the previous ones.  A series'
first chunk therefore starts from the prior itself: combining the prior
with a chunk's information about its first state, (I + P0 J)^-1 with J of
order 1/R, loses every digit (errors of order 1 at 1e-9 noise before this
was done); the sequential filter is checked as well."""
import numpy as np
import pytest

import conditioning_cases as CC
from oracle import exact

pytestmark = pytest.mark.gpu

OPTS = (dict(), dict(single_chunk=1), dict(chunk_min=4, chunk_target=8))


def _plan(lib, ts, te, y, yerr, **opt):
    return lib.Plan(np.array([0, len(ts)], dtype=np.int64), ts, te, y, yerr, **opt)


def _grad_err(g, ref):
    den = np.maximum(np.abs(ref), 1e-3 * np.max(np.abs(ref)))
    return np.max(np.abs(g - ref) / den)


@pytest.mark.parametrize("instantaneous", [True, False])
def test_nearly_noise_free_single_term(lib, instantaneous):
    for noise in (1e-5, 1e-7, 1e-9):
        for omega0 in (0.5, 5.0):
            ts, te, y, yerr, sig, w0, q = CC.smooth(31, 40, noise, omega0, instantaneous)
            Le = exact.loglik(ts, te, y, yerr, sig, w0, q, 0.0, dps=80)
            errs = []
            for opt in OPTS:
                plan = _plan(lib, ts, te, y, yerr, **opt)
                ll, st = plan.loglik(sig[None], w0[None], q[None], np.zeros(1), status=True)
                assert int(st.cpu()[0]) == 0
                errs.append(abs(float(ll.cpu()[0]) - Le) / abs(Le))
            pl = float(plan.plain_loglik(sig[None], w0[None], q[None], np.zeros(1)).cpu()[0])
            errs.append(abs(pl - Le) / abs(Le))
            print(instantaneous, noise, omega0, Le, errs)
            assert max(errs) < 1e-9, (noise, omega0, errs)


def test_nearly_noise_free_two_instruments(lib):
    for seed in (21, 22):
        for noise in (1e-5, 1e-9):
            ts, te, y, yerr, sig, w0, q = CC.two_instruments(seed, 50, noise)
            Le = exact.loglik(ts, te, y, yerr, sig, w0, q, 0.0, dps=80)
            for opt in OPTS:
                plan = _plan(lib, ts, te, y, yerr, **opt)
                ll = float(plan.loglik(sig[None], w0[None], q[None], np.zeros(1)).cpu()[0])
                print(seed, noise, opt, plan.stats()["max_slots"], abs(ll - Le) / abs(Le))
                assert abs(ll - Le) < 1e-9 * abs(Le)


@pytest.mark.parametrize("instantaneous,omega0", [(True, 0.5), (False, 5.0)])
def test_nearly_noise_free_gradient(lib, instantaneous, omega0):
    ts, te, y, yerr, sig, w0, q = CC.smooth(31, 40, 1e-7, omega0, instantaneous)
    gref = exact.loglik_grad_fd(ts, te, y, yerr, sig, w0, q, 0.0, dps=80)
    for opt in (dict(), dict(chunk_min=4, chunk_target=8)):
        plan = _plan(lib, ts, te, y, yerr, **opt)
        _, g = plan.loglik_grad(sig[None], w0[None], q[None], np.zeros(1))
        g = g.cpu().numpy()[0]
        # zero jitter: its derivative is exactly 0 (the likelihood is even in it)
        assert g[-1] == 0.0
        e = _grad_err(g[:-1], gref[:-1])
        print(instantaneous, omega0, opt, e)
        assert e < 1e-6


@pytest.mark.parametrize("instantaneous", [True, False])
def test_nearly_noise_free_smoother(lib, instantaneous):
    """Posterior of the measured quantities at the data, against the
    high-precision dense posterior, relative to the posterior itself: means
    within 1e-9 of the posterior standard deviation, variances within 1e-9
    relative (the smoother takes them in disturbance form, of order R here,
    far below the predicted variances).  At the test times, where the
    posterior comes from the predicted moments and the adjoint pair, means
    within 1e-9 of the posterior standard deviation and variances within
    1e-5 relative: their absolute error is that of the predicted covariance,
    a few ulp of the prior variance, against posterior variances down to
    1e-10 of it."""
    for noise in (1e-3, 1e-5, 1e-7):
        ts, te, y, yerr, sig, w0, q = CC.smooth(31, 40, noise, 0.5, instantaneous)
        tt = np.sort(np.concatenate([np.linspace(ts[0] - 0.2, te[-1] + 0.2, 15), 0.5 * (ts[5:9] + te[6:10])]))
        md_e, vd_e = exact.posterior_data(ts, te, y, yerr, sig, w0, q, 0.0, dps=60)
        mt_e, vt_e = exact.posterior_test(ts, te, y, yerr, sig, w0, q, tt, 0.0, dps=60)
        for opt in (dict(), dict(chunk_min=4, chunk_target=8)):
            plan = _plan(lib, ts, te, y, yerr, **opt)
            o = plan.smooth(sig[None], w0[None], q[None], np.zeros(1), np.array([0, len(tt)], dtype=np.int64), tt)
            md, vd, mt, vt = (o[k].cpu().numpy() for k in ("mean_data", "var_data", "mean_test", "var_test"))
            errs = (np.max(np.abs(md - md_e) / np.sqrt(vd_e)), np.max(np.abs(vd - vd_e) / vd_e),
                    np.max(np.abs(mt - mt_e) / np.sqrt(vt_e)), np.max(np.abs(vt - vt_e) / vt_e))
            print(instantaneous, noise, opt, errs)
            assert errs[0] < 1e-9 and errs[1] < 1e-9 and errs[2] < 1e-9, errs
            assert errs[3] < 1e-5, errs
