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
