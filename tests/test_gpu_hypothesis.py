"""Hypothesis-fuzzed tiny problems on the GPU against the dense oracle
(quadrature + Cholesky, Sec. 3.1 and Sec. 2.4): exposure sets with equal
times, zero-length exposures and overlaps up to three deep (the strategies of
interval_strategies.py), one or two SHO terms with random hyperparameters,
with and without jitter, under two chunkings, and the square-root filter
(sequential and split in time).
Log-likelihood within 1e-9 of max(1, |L|), gradient within 1e-6 (relative
to max(|g_i|, 1e-3 max|g|)).
The examples are derandomized: every run tries the same ones."""
import numpy as np
import pytest
from hypothesis import HealthCheck, given, settings, strategies as st

import interval_strategies as IS
from oracle import dense

pytestmark = pytest.mark.gpu


def _grad_err(g, ref):
    den = np.maximum(np.abs(ref), 1e-3 * np.max(np.abs(ref)))
    return np.max(np.abs(g - ref) / den)


@settings(max_examples=40, derandomize=True, deadline=None, suppress_health_check=[HealthCheck.function_scoped_fixture])
@given(ser=IS.exposure_series(max_instruments=3, max_per_instrument=5),
       M=st.integers(1, 2),
       seed=st.integers(0, 2 ** 31 - 1),
       jitter=st.sampled_from([0.0, 0.05]),
       chunked=st.booleans())
def test_fuzzed_tiny_problems_match_dense(lib, ser, M, seed, jitter, chunked):
    ts, te, _ = ser
    n = len(ts)
    if n == 0:
        return
    rng = np.random.default_rng(seed)
    sig = np.exp(rng.uniform(np.log(0.3), np.log(2.0), M))
    w0 = np.exp(rng.uniform(np.log(0.5), np.log(50.0), M))
    q = np.exp(rng.uniform(np.log(0.3), np.log(20.0), M))
    yerr = rng.uniform(0.05, 0.3, n)
    y = rng.normal(0.0, 1.0, n)
    L, g_ref = dense.loglik_grad(ts, te, y, yerr, sig, w0, q, jitter)
    opt = dict(chunk_min=1, chunk_target=2) if chunked else dict()
    plan = lib.Plan(np.array([0, n], dtype=np.int64), ts, te, y, yerr, **opt)
    ll, g, st_ = plan.loglik_grad(sig[None], w0[None], q[None], np.array([jitter]), status=True)
    ll, g = float(ll.cpu().numpy()[0]), g.cpu().numpy()[0]
    assert int(st_.cpu().numpy()[0]) == 0
    assert abs(ll - L) <= 1e-9 * max(1.0, abs(L)), (ll, L)
    ls = float(plan.loglik_sqrt(sig[None], w0[None], q[None], np.array([jitter]), check=True).cpu().numpy()[0])
    assert abs(ls - L) <= 1e-9 * max(1.0, abs(L)), (ls, L)
    ls = float(plan.loglik_sqrt_split(sig[None], w0[None], q[None], np.array([jitter]), check=True).cpu().numpy()[0])
    assert abs(ls - L) <= 1e-9 * max(1.0, abs(L)), (ls, L)
    if jitter == 0.0:
        assert g[-1] == 0.0
    assert _grad_err(g, g_ref) < 1e-6, (g, g_ref)
