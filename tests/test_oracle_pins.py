"""Pins of the oracle against what the paper and the mathematics fix
(closed forms, library routines, invariants, brute force).  CPU only."""
import math

import mpmath as mp
import numpy as np
import pytest
import scipy.integrate as si
import scipy.linalg as sl

from oracle import dense, kalman, sho
import workloads as W

QS = [0.3, 0.5, 0.5 + 1e-9, 0.5 - 1e-9, 1 / math.sqrt(2), 30.0]


# ---------------------------------------------------------------------------
# kernel and state-space model (Appendix B)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("q", [0.3, 0.5, 1 / math.sqrt(2), 3.0, 30.0])
def test_kernel_equals_ssm_covariance(q):
    """k(Delta) = H Pinf Phi(Delta)^T H^T (Sec. 2.2, kernel from the SSM) with
    Phi from scipy's matrix exponential."""
    s, w0 = 1.3, 2.0
    F, L, Qc, Pinf = sho.ssm(s, w0, q)
    for d in [0.0, 1e-4, 0.03, 0.5, 2.0, 9.0]:
        k_ssm = (Pinf @ sl.expm(F * d).T)[0, 0]
        assert abs(sho.kernel(d, s, w0, q) - k_ssm) <= 1e-13 * s * s  # expm rounding


@pytest.mark.parametrize("q", [0.4, 1 / math.sqrt(2), 4.0])
def test_kernel_is_fourier_dual_of_psd(q):
    """k(Delta) = (1/2pi) int S(omega) e^{i omega Delta} d omega (Sec. 2.2.1,
    Wiener-Khinchin; PSD of Appendix B)."""
    s, w0 = 0.8, 1.5
    for d in [0.0, 0.7, 2.5]:
        f = lambda om: sho.psd(om, s, w0, q) * math.cos(om * d) / math.pi
        val = si.quad(f, 0, np.inf, limit=400, epsabs=1e-13, epsrel=1e-12)[0]
        assert abs(val - sho.kernel(d, s, w0, q)) < 1e-9


def test_kernel_grad_matches_finite_differences():
    s, w0 = 0.7, 5.0
    u = np.array([0.02, 0.3, 1.0, 4.0])
    for q in [0.3, 0.5, 2.0]:
        g = sho.kernel_grad(u, s, w0, q)
        for i, base in enumerate((s, w0, q)):
            h = 1e-5 * base
            args_p = [s, w0, q]
            args_m = [s, w0, q]
            args_p[i] += h
            args_m[i] -= h
            fd = (sho.kernel(u, *args_p) - sho.kernel(u, *args_m)) / (2 * h)
            assert np.allclose(g[i], fd, rtol=1e-7, atol=1e-12)


@pytest.mark.parametrize("q", [0.3, 0.5, 1 / math.sqrt(2), 30.0])
def test_stationary_covariance_solves_lyapunov(q):
    """F Pinf + Pinf F^T + L Qc L^T = 0 (Sec. 2.2.2; Appendix B)."""
    F, L, Qc, Pinf = sho.ssm(0.9, 3.0, q)
    P = sl.solve_continuous_lyapunov(F, -(L * Qc) @ L.T)
    assert np.allclose(P, Pinf, rtol=1e-12, atol=1e-13 * np.max(Pinf))


# ---------------------------------------------------------------------------
# Appendix B closed forms (mpmath) vs library routines and quadrature
# ---------------------------------------------------------------------------

def _augmented(s, w0, q):
    F, L, Qc, Pinf = sho.ssm(s, w0, q)
    Fa = np.zeros((3, 3))
    Fa[:2, :2] = F
    Fa[2, 0] = 1.0
    La = np.array([[0.0], [1.0], [0.0]])
    return Fa, La, Qc


@pytest.mark.parametrize("x", [0.19, 1.4])
@pytest.mark.parametrize("q", [0.4, 1 / math.sqrt(2), 30.0])
def test_closed_forms_match_van_loan(x, q):
    """Appendix B closed forms == the Van Loan block exponential of the
    augmented model (Appendix B, augmented noise from one exponential).
    Only short steps: the single exponential loses digits as omega0*dt
    grows (about 6 digits by omega0*dt = 6), the instability the paper notes
    for that route."""
    s, w0 = 1.1, 2.0
    dt = x / w0
    cf = sho.closed_forms(s, w0, q, dt)
    Fa, La, Qc = _augmented(s, w0, q)
    n = 3
    Mvl = np.zeros((2 * n, 2 * n))
    Mvl[:n, :n] = -Fa
    Mvl[:n, n:] = (La * Qc) @ La.T
    Mvl[n:, n:] = Fa.T
    E = sl.expm(Mvl * dt)
    F3 = E[n:, n:]
    G2 = E[:n, n:]
    Qa = F3.T @ G2
    Phia = sl.expm(Fa * dt)
    scale_q = np.max(np.abs(Qa))
    assert np.allclose(Phia[:2, :2], cf["Phi"], rtol=0, atol=1e-12)
    assert np.allclose(Phia[2, :2], cf["Phibar"][0], rtol=0, atol=1e-12)
    assert np.allclose(Qa[:2, :2], cf["Qk"], rtol=0, atol=1e-11 * scale_q)
    assert np.allclose(Qa[:2, 2], cf["q12"], rtol=0, atol=1e-11 * scale_q)
    assert abs(Qa[2, 2] - cf["q22"]) <= 1e-11 * scale_q


@pytest.mark.parametrize("q", [0.4, 1 / math.sqrt(2), 7.0])
def test_closed_forms_match_defining_integrals(q):
    """Phibar = int Phi, Q12 = first column of int Phi L Qc L^T Phibar^T,
    Q22 = first element of int Phibar L Qc L^T Phibar^T (Sec. 3.2 and
    Appendix B), by adaptive quadrature with Phi from expm."""
    s, w0, dt = 0.9, 1.7, 0.8
    F, L, Qc, Pinf = sho.ssm(s, w0, q)
    cf = sho.closed_forms(s, w0, q, dt)
    Phi = lambda t: sl.expm(F * t)
    Phibar = lambda t: np.array([[si.quad(lambda u: Phi(u)[i, j], 0, t, epsabs=1e-14)[0] for j in range(2)]
                                 for i in range(2)])
    pb = Phibar(dt)
    assert np.allclose(pb, cf["Phibar"], atol=1e-12)
    q12 = [si.quad(lambda t: Phi(t)[i, 1] * Qc * Phibar(t)[0, 1], 0, dt, epsabs=1e-13)[0] for i in range(2)]
    assert np.allclose(q12, cf["q12"], atol=1e-10)
    q22 = si.quad(lambda t: Phibar(t)[0, 1] ** 2 * Qc, 0, dt, epsabs=1e-14)[0]
    assert abs(q22 - cf["q22"]) < 1e-11
    Qk = np.array([[si.quad(lambda t: (Phi(t) @ L @ L.T @ Phi(t).T)[i, j] * Qc, 0, dt, epsabs=1e-13)[0]
                    for j in range(2)] for i in range(2)])
    assert np.allclose(Qk, cf["Qk"], atol=1e-10)


# ---------------------------------------------------------------------------
# the oracle's discretisation (Taylor + doubling, long double)
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("q", QS)
def test_oracle_discretisation_matches_closed_forms(q):
    s, w0 = 1.3, 2.0
    Pinf = np.diag([s * s, s * s * w0 * w0])
    for x in [0.0, 1e-6, 1e-4, 1e-2, 0.1, 0.5, 1.0, 3.0, 7.0, 20.0, 100.0, 1e3]:
        dt = x / w0
        phi, qq = kalman.term_discretise(w0, q, s, dt)
        if x == 0:
            assert np.array_equal(phi, np.eye(3)) and np.all(qq == 0)
            continue
        dps = 200 if abs(q - 0.5) < 1e-6 else 80
        cf = sho.closed_forms(s, w0, q, dt, dps=dps)
        # transition in the scaled frame (x, xdot/w0) relative to O(1)
        T = np.diag([1.0, 1.0 / w0])
        Ti = np.diag([1.0, w0])
        assert np.allclose(T @ phi[:2, :2] @ Ti, T @ cf["Phi"] @ Ti, rtol=0, atol=3e-16)
        # process noise relative to Pinf
        assert np.allclose(qq[:2, :2] / np.sqrt(np.outer(np.diag(Pinf), np.diag(Pinf))),
                           cf["Qk"] / np.sqrt(np.outer(np.diag(Pinf), np.diag(Pinf))), rtol=0, atol=3e-16)
        # integrated quantities: entry-wise relative (they do not vanish)
        assert np.allclose(phi[2, :2], cf["Phibar"][0], rtol=3e-15, atol=0)
        assert np.allclose(qq[:2, 2], cf["q12"], rtol=5e-14, atol=1e-300 + 1e-15 * np.max(np.abs(cf["q12"])))
        assert abs(qq[2, 2] - cf["q22"]) <= 3e-15 * abs(cf["q22"])


def test_process_noise_identity():
    """Q_k = Pinf - A Pinf A^T (Sec. 2.2.2)."""
    for q in [0.3, 0.5, 2.0]:
        s, w0 = 0.7, 4.0
        Pinf = np.diag([s * s, s * s * w0 * w0])
        for dt in [1e-3, 0.2, 3.0]:
            phi, qq = kalman.term_discretise(w0, q, s, dt)
            A = phi[:2, :2]
            assert np.allclose(qq[:2, :2], Pinf - A @ Pinf @ A.T, rtol=0, atol=1e-14 * s * s * w0 * w0)


def test_small_step_leading_terms():
    """Exact leading terms for small steps: Q_k[0,0] ~ Qc dt^3/3,
    q12 ~ (Qc dt^4/8, Qc dt^3/6), q22 ~ Qc dt^5/20."""
    s, w0, q = 1.0, 3.0, 2.0
    Qc = 2 * w0 ** 3 * s * s / q
    dt = 1e-5
    phi, qq = kalman.term_discretise(w0, q, s, dt)
    assert abs(qq[0, 0] / (Qc * dt ** 3 / 3) - 1) < 1e-4
    assert abs(qq[0, 2] / (Qc * dt ** 4 / 8) - 1) < 1e-4
    assert abs(qq[1, 2] / (Qc * dt ** 3 / 6) - 1) < 1e-4
    assert abs(qq[2, 2] / (Qc * dt ** 5 / 20) - 1) < 1e-4


@pytest.mark.parametrize("q", [0.4, 1 / math.sqrt(2), 30.0])
def test_integrated_variance_grows_with_psd_at_zero(q):
    """q22 grows linearly with slope S(0) (Appendix B remark; PSD at omega = 0)."""
    s, w0 = 1.2, 5.0
    dt = 400.0 / w0 * max(q, 1)
    h = 1.0
    _, q1 = kalman.term_discretise(w0, q, s, dt)
    _, q2 = kalman.term_discretise(w0, q, s, dt + h)
    slope = (q2[2, 2] - q1[2, 2]) / h
    assert abs(slope / sho.psd(0.0, s, w0, q) - 1) < 1e-9


# ---------------------------------------------------------------------------
# dense integrated covariance vs the Appendix A closed forms
# ---------------------------------------------------------------------------

def _celerite_integrated(a, b, c, d, delta, lag):
    """Appendix A: exposure-averaged celerite kernel for equal exposures
    delta at midpoint lag (non-overlapping, overlapping and diagonal)."""
    with mp.workdps(50):
        a, b, c, d, delta, lag = (mp.mpf(v) for v in (a, b, c, d, delta, lag))
        C1 = a * c * c - a * d * d + 2 * b * c * d
        C2 = b * c * c - b * d * d - 2 * a * c * d
        den = delta ** 2 * (c * c + d * d) ** 2
        A = (2 * C1 * (mp.cosh(c * delta) * mp.cos(d * delta) - 1) - 2 * C2 * mp.sinh(c * delta) * mp.sin(d * delta)) / den
        B = (2 * C2 * (mp.cosh(c * delta) * mp.cos(d * delta) - 1) + 2 * C1 * mp.sinh(c * delta) * mp.sin(d * delta)) / den
        if lag == 0:
            v = 2 * ((a * c + b * d) * (c * c + d * d) * delta - C1
                     + mp.exp(-c * delta) * (C1 * mp.cos(d * delta) + C2 * mp.sin(d * delta))) / den
            return float(v)
        base = A * mp.exp(-c * lag) * mp.cos(d * lag) + B * mp.exp(-c * lag) * mp.sin(d * lag)
        if lag >= delta:
            return float(base)
        extra = 2 * ((a * c + b * d) * (c * c + d * d) * (delta - lag)
                     - C1 * mp.sinh(c * delta - c * lag) * mp.cos(d * delta - d * lag)
                     + C2 * mp.cosh(c * delta - c * lag) * mp.sin(d * delta - d * lag)) / (delta * (c * c + d * d)) ** 2
        return float(base + extra)


@pytest.mark.parametrize("q", [1 / math.sqrt(2), 5.0])
def test_dense_covariance_matches_appendix_a(q):
    s, w0 = 1.1, 3.0
    eta = math.sqrt(1 - 1 / (4 * q * q))
    a, b, c, d = s * s, s * s / (2 * eta * q), w0 / (2 * q), eta * w0
    delta = 0.4
    mids = np.array([0.0, 0.13, 0.4, 0.9, 2.5])
    ts = mids - delta / 2
    te = mids + delta / 2
    K = dense.covariance(ts, te, [s], [w0], [q])
    for i in range(len(mids)):
        for j in range(len(mids)):
            ref = _celerite_integrated(a, b, c, d, delta, abs(mids[i] - mids[j]))
            assert abs(K[i, j] - ref) < 1e-14 * s * s, (i, j)


def test_dense_instantaneous_limit():
    """delta -> 0: the integrated covariance tends to k(t_i - t_j), O(delta^2)."""
    s, w0, q = 1.0, 2.0, 3.0
    mids = np.array([0.0, 0.3, 1.1])
    for delta in [1e-2, 1e-3]:
        K = dense.covariance(mids - delta / 2, mids + delta / 2, [s], [w0], [q])
        ref = sho.kernel(mids[:, None] - mids[None, :], s, w0, q)
        assert np.max(np.abs(K - ref)) < 2 * (w0 * delta) ** 2
    K0 = dense.covariance(mids, mids, [s], [w0], [q])
    assert np.allclose(K0, sho.kernel(mids[:, None] - mids[None, :], s, w0, q), rtol=0, atol=1e-15)


# ---------------------------------------------------------------------------
# sequential Kalman oracle == dense integrated GP
# ---------------------------------------------------------------------------

def _both(b, idx=0):
    s = b.series(idx)
    Ld = dense.loglik(s["ts"], s["te"], s["y"], s["yerr"], s["sigma"], s["omega0"], s["quality"], s["jitter"])
    Lk = kalman.loglik(s["ts"], s["te"], s["y"], s["yerr"], s["sigma"], s["omega0"], s["quality"], s["jitter"])
    return Ld, Lk


@pytest.mark.parametrize("make", [W.small_single, W.small_multi])
def test_kalman_equals_dense_validation_scenarios(make):
    """The paper reports agreement to 1e-14 for these two scenarios."""
    Ld, Lk = _both(make())
    assert abs(Ld - Lk) <= 1e-12 * abs(Ld)


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_kalman_equals_dense_random(seed):
    b = W.random_small_batch(seed, B=3, n_lo=5, n_hi=40, M=2, J=3)
    for i in range(b.n_series):
        Ld, Lk = _both(b, i)
        assert abs(Ld - Lk) <= 1e-11 * max(1.0, abs(Ld)), (seed, i, Ld, Lk)


def test_single_exposure_closed_form():
    """N = 1: L = -1/2 (log 2 pi (K11 + r) + y^2 / (K11 + r)), K11 the
    Appendix A diagonal."""
    s, w0, q = 1.0, 2.0, 1.5
    eta = math.sqrt(1 - 1 / (4 * q * q))
    a, b, c, d = s * s, s * s / (2 * eta * q), w0 / (2 * q), eta * w0
    delta, y, r = 0.7, 0.37, 0.04
    K11 = _celerite_integrated(a, b, c, d, delta, 0.0)
    ref = -0.5 * (math.log(2 * math.pi * (K11 + r)) + y * y / (K11 + r))
    L = kalman.loglik([1.0], [1.0 + delta], [y], [math.sqrt(r)], [s], [w0], [q])
    assert abs(L - ref) < 1e-14


def test_zero_length_exposures_reduce_to_textbook_gp():
    """All exposures instantaneous: the textbook GP with K_ij = k(t_i - t_j)
    (Sec. 2.1), written out with the kernel and a Cholesky."""
    rng = np.random.default_rng(7)
    t = np.sort(rng.uniform(0, 3, 25))
    y = rng.normal(size=25)
    yerr = rng.uniform(0.1, 0.3, 25)
    sig, w0, q = [1.0, 0.5], [2.0, 9.0], [0.8, 0.4]
    K = sum(sho.kernel(t[:, None] - t[None, :], sig[m], w0[m], q[m]) for m in range(2))
    C = np.linalg.cholesky(K + np.diag(yerr ** 2))
    al = np.linalg.solve(C.T, np.linalg.solve(C, y))
    ref = -0.5 * y @ al - np.sum(np.log(np.diag(C))) - 0.5 * 25 * math.log(2 * math.pi)
    L = kalman.loglik(t, t, y, yerr, sig, w0, q)
    assert abs(L - ref) < 1e-12 * abs(ref)


def test_labelling_invariance():
    """Any valid instrument labelling, and unused extra integrators, give the
    same likelihood."""
    b = W.small_multi()
    s = b.series(0)
    args = (s["ts"], s["te"], s["y"], s["yerr"], s["sigma"], s["omega0"], s["quality"], 0.02)
    slots, J = kalman.greedy_slots(s["ts"], s["te"])
    L0 = kalman.loglik(*args)
    # relabel: reverse label order
    L1 = kalman.loglik(*args, slots=(J - 1 - slots))
    # put each exposure on its own label when possible: labels 0..J+1 cycling
    L2 = kalman.loglik(*args, extra_slots=2)
    assert abs(L1 - L0) < 1e-13 * abs(L0)
    assert abs(L2 - L0) < 1e-13 * abs(L0)
    with pytest.raises(kalman.OracleError):
        kalman.loglik(*args, slots=np.zeros_like(slots))  # self-overlapping label


def test_p0_integrator_block_irrelevant():
    """The integrators are reset before use, so the likelihood does not
    depend on P0's integrator block: first exposure later than a long
    instantaneous prefix gives the same value as the dense GP."""
    ts = np.array([0.0, 0.1, 0.3, 0.35])
    te = np.array([0.0, 0.2, 0.3, 0.5])
    y = np.array([0.2, -0.1, 0.4, 0.3])
    yerr = np.full(4, 0.1)
    Ld = dense.loglik(ts, te, y, yerr, [1.0], [5.0], [1.0])
    Lk = kalman.loglik(ts, te, y, yerr, [1.0], [5.0], [1.0])
    assert abs(Ld - Lk) < 1e-13 * abs(Ld)


# ---------------------------------------------------------------------------
# smoother and prediction vs the dense posterior
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("make", [W.small_single, W.small_multi])
def test_smoother_equals_dense_posterior(make):
    b = make()
    s = b.series(0)
    args = (s["ts"], s["te"], s["y"], s["yerr"], s["sigma"], s["omega0"], s["quality"], 0.01)
    md, vd, mt, vt = dense.posterior(*args, t_test=b.t_test)
    L, mt2, vt2, md2, vd2 = kalman.smooth(*args, t_test=b.t_test)
    k0 = float(np.sum(np.asarray(s["sigma"]) ** 2))
    assert np.max(np.abs(md - md2)) < 1e-10 * math.sqrt(k0)
    assert np.max(np.abs(vd - vd2)) < 1e-10 * k0
    assert np.max(np.abs(mt - mt2)) < 1e-10 * math.sqrt(k0)
    assert np.max(np.abs(vt - vt2)) < 1e-10 * k0


def test_smoother_test_times_at_events_and_ties():
    b = W.random_small_batch(5, B=1, n_lo=30, n_hi=30, M=2, J=3)
    s = b.series(0)
    tt = np.concatenate([s["ts"][:5], s["te"][-5:], [s["ts"][0] - 1.0, s["te"].max() + 0.5]])
    args = (s["ts"], s["te"], s["y"], s["yerr"], s["sigma"], s["omega0"], s["quality"], s["jitter"])
    md, vd, mt, vt = dense.posterior(*args, t_test=tt)
    L, mt2, vt2, md2, vd2 = kalman.smooth(*args, t_test=tt)
    assert np.max(np.abs(mt - mt2)) < 1e-9
    assert np.max(np.abs(vt - vt2)) < 1e-9
    assert np.max(np.abs(md - md2)) < 1e-9
    assert np.max(np.abs(vd - vd2)) < 1e-9


def test_prediction_far_from_data_reverts_to_prior():
    b = W.small_multi()
    s = b.series(0)
    args = (s["ts"], s["te"], s["y"], s["yerr"], s["sigma"], s["omega0"], s["quality"], 0.0)
    far = np.array([-1e3, 1e3])
    L, mt, vt, _, _ = kalman.smooth(*args, t_test=far)
    assert np.allclose(mt, 0.0, atol=1e-12)
    assert np.allclose(vt, np.sum(np.asarray(s["sigma"]) ** 2), rtol=1e-12)


def test_smoother_accuracy_near_coincident_starts():
    """The oracle's smoother (the RTS recursion of Sec. 3.2.2, long double)
    inverts the predicted covariance, which is nearly singular where two
    exposures start 3 ms apart: against the dense posterior (Sec. 2.1) its
    smoothed variances just before the pair stay within 1e-6 of the prior
    variance, and away from it within 1e-12 -- the accuracy the full-size
    smoother comparison allows for."""
    rng = np.random.default_rng(3)
    s1, e1 = W.place_slot(rng, 1.0, rng.uniform(5, 15, 30) / 1440.0)
    s2, e2 = W.place_slot(rng, 1.0, rng.uniform(5, 15, 30) / 1440.0)
    j = int(np.argmin(np.abs(s2 - s1[15])))
    length = e2[j] - s2[j]
    s2[j] = s1[15] + 3e-3 / 86400.0
    e2[j] = s2[j] + length
    ts, te = np.concatenate([s1, s2]), np.concatenate([e1, e2])
    o = np.argsort(ts, kind="stable")
    ts, te = ts[o], te[o]
    sig, w0, q = [1.0, 0.5], [2 * np.pi / 0.2, 2 * np.pi * 1440 / 5], [1 / np.sqrt(2), 30.0]
    yerr = np.full(len(ts), 0.2)
    y = rng.normal(size=len(ts)) * 0.5
    _, vd_dense, _, _ = dense.posterior(ts, te, y, yerr, sig, w0, q, 0.0)
    _, _, _, _, vd = kalman.smooth(ts, te, y, yerr, sig, w0, q, 0.0)
    err = np.abs(vd - vd_dense) / 1.25
    p = int(np.argmin(np.diff(ts)))
    assert np.diff(ts)[p] * 86400.0 < 0.01
    away = np.r_[err[:p - 12], err[p + 3:]]
    assert err.max() < 1e-6 and away.max() < 1e-12, (err.max(), away.max())


# ---------------------------------------------------------------------------
# component-wise prediction (Appendix C, component-wise predictive means and
# variances)
# ---------------------------------------------------------------------------

def test_dense_terms_reconstruct_the_total():
    """The appendix's reconstruction: the total mean is the sum of the term
    means, and the total variance is the sum of the term variances minus the
    cross terms K_{m,*}^T K_y^-1 K_{l,*} over m != l (K_y: data covariance
    with the noise)."""
    b = W.random_small_batch(8, B=1, n_lo=40, n_hi=40, M=3, J=2)
    s = b.series(0)
    tt = np.linspace(s["ts"].min() - 0.2, s["te"].max() + 0.2, 17)
    args = (s["ts"], s["te"], s["y"], s["yerr"], s["sigma"], s["omega0"], s["quality"], s["jitter"])
    _, _, mt, vt = dense.posterior(*args, t_test=tt)
    tm, tv, Ks = dense.posterior_terms(*args, t_test=tt)
    K = dense.covariance(s["ts"], s["te"], s["sigma"], s["omega0"], s["quality"])
    Ky = K + np.diag(np.asarray(s["yerr"]) ** 2 + s["jitter"] ** 2)
    cross = np.zeros(len(tt))
    for m in range(3):
        for l in range(3):
            if m != l:
                cross += np.sum(Ks[m] * np.linalg.solve(Ky, Ks[l]), axis=0)
    assert np.max(np.abs(tm.sum(axis=1) - mt)) < 1e-12
    assert np.max(np.abs(tv.sum(axis=1) - cross - vt)) < 1e-12


def test_dense_single_term_equals_total():
    b = W.random_small_batch(9, B=1, n_lo=30, n_hi=30, M=1, J=2)
    s = b.series(0)
    tt = np.linspace(s["ts"].min() - 0.1, s["te"].max() + 0.1, 11)
    args = (s["ts"], s["te"], s["y"], s["yerr"], s["sigma"], s["omega0"], s["quality"], s["jitter"])
    _, _, mt, vt = dense.posterior(*args, t_test=tt)
    tm, tv, _ = dense.posterior_terms(*args, t_test=tt)
    assert np.max(np.abs(tm[:, 0] - mt)) < 1e-13
    assert np.max(np.abs(tv[:, 0] - vt)) < 1e-13


def test_kalman_terms_equal_dense_terms():
    """H^m applied to the smoothed state (Kalman oracle) against the dense
    component posterior, with test times before, between, at and after the
    events, two terms and overlapping exposures."""
    b = W.random_small_batch(5, B=1, n_lo=30, n_hi=30, M=2, J=3)
    s = b.series(0)
    tt = np.concatenate([s["ts"][:4], s["te"][-4:], np.linspace(s["ts"].min() - 0.5, s["te"].max() + 0.5, 23)])
    args = (s["ts"], s["te"], s["y"], s["yerr"], s["sigma"], s["omega0"], s["quality"], s["jitter"])
    tm, tv, _ = dense.posterior_terms(*args, t_test=tt)
    out = kalman.smooth(*args, t_test=tt, terms=True)
    tm2, tv2 = out[5], out[6]
    assert tm2.shape == (len(tt), 2)
    assert np.max(np.abs(tm - tm2)) < 1e-9
    assert np.max(np.abs(tv - tv2)) < 1e-9
    # the totals are unchanged by asking for the terms
    L, mt, vt, _, _ = kalman.smooth(*args, t_test=tt)
    assert np.array_equal(out[1], mt) and np.array_equal(out[2], vt)


def test_terms_far_from_data_revert_to_their_priors():
    b = W.small_multi()
    s = b.series(0)
    args = (s["ts"], s["te"], s["y"], s["yerr"], s["sigma"], s["omega0"], s["quality"], 0.0)
    out = kalman.smooth(*args, t_test=np.array([-1e3, 1e3]), terms=True)
    sig = np.atleast_1d(np.asarray(s["sigma"], dtype=np.float64))
    assert np.allclose(out[5], 0.0, atol=1e-12)
    assert np.allclose(out[6], np.broadcast_to(sig ** 2, out[6].shape), rtol=1e-12)


# ---------------------------------------------------------------------------
# gradients
# ---------------------------------------------------------------------------

def test_dense_gradient_matches_fd_of_dense():
    b = W.random_small_batch(9, B=1, n_lo=25, n_hi=25, M=2, J=2)
    s = b.series(0)
    sig, w0, q, jit = s["sigma"], s["omega0"], s["quality"], 0.05
    L, g = dense.loglik_grad(s["ts"], s["te"], s["y"], s["yerr"], sig, w0, q, jit)
    th = np.concatenate([sig, w0, q, [jit]])
    M = len(sig)
    K = None
    for i in range(len(th)):
        h = 1e-6 * abs(th[i])
        tp, tm = th.copy(), th.copy()
        tp[i] += h
        tm[i] -= h
        f = lambda t: dense.loglik(s["ts"], s["te"], s["y"], s["yerr"], t[:M], t[M:2 * M], t[2 * M:3 * M], t[3 * M])
        fd = (f(tp) - f(tm)) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * max(abs(g[i]), 1e-3 * np.max(np.abs(g))), i


def test_dense_gradient_matches_fd_of_kalman():
    b = W.small_multi()
    s = b.series(0)
    args = (s["ts"], s["te"], s["y"], s["yerr"], s["sigma"], s["omega0"], s["quality"], 0.03)
    L, g = dense.loglik_grad(*args)
    gfd = kalman.loglik_grad_fd(*args)
    den = np.maximum(np.abs(g), 1e-3 * np.max(np.abs(g)))
    assert np.max(np.abs(g - gfd) / den) < 1e-7


# ---------------------------------------------------------------------------
# labels
# ---------------------------------------------------------------------------

def test_greedy_labels_use_overlap_depth_and_never_self_overlap():
    rng = np.random.default_rng(3)
    for trial in range(50):
        n = int(rng.integers(1, 40))
        ts = np.sort(rng.uniform(0, 1, n))
        te = ts + rng.uniform(0, 0.2, n)
        inst = rng.uniform(size=n) < 0.1
        te[inst] = ts[inst]
        # depth by brute force: max number of windows open at any start time
        depth = 0
        for t in ts[~inst]:
            depth = max(depth, int(np.sum((ts <= t) & (te > t))))
        if depth > 8:
            with pytest.raises(kalman.OracleError):
                kalman.greedy_slots(ts, te)
            continue
        slots, J = kalman.greedy_slots(ts, te)
        assert np.all(slots[inst] == -1)
        assert J == depth
        for j in range(J):
            sel = np.where(slots == j)[0]
            order = sel[np.argsort(ts[sel])]
            assert np.all(te[order[:-1]] <= ts[order[1:]])


# ---------------------------------------------------------------------------
# real (exponential) terms: the celerite term of Appendix A with b = d = 0,
# sigma^2 exp(-c |tau|), a one-state model; and the Matern-3/2 kernel as the
# SHO term at Q = 1/2
# ---------------------------------------------------------------------------

def test_dense_real_term_matches_appendix_a():
    s, c = 0.8, 2.3
    delta = 0.4
    mids = np.array([0.0, 0.13, 0.4, 0.9, 2.5])
    K = dense.covariance(mids - delta / 2, mids + delta / 2, [s], [c], [1.0], kinds=["real"])
    for i in range(len(mids)):
        for j in range(len(mids)):
            ref = _celerite_integrated(s * s, 0.0, c, 0.0, delta, abs(mids[i] - mids[j]))
            assert abs(K[i, j] - ref) < 1e-14 * s * s, (i, j)


def test_real_term_single_exposure_closed_form():
    """N = 1 with a real term: K11 from Appendix A at b = d = 0."""
    s, c = 1.3, 0.7
    delta, y, r = 0.9, -0.21, 0.03
    K11 = _celerite_integrated(s * s, 0.0, c, 0.0, delta, 0.0)
    ref = -0.5 * (math.log(2 * math.pi * (K11 + r)) + y * y / (K11 + r))
    L = kalman.loglik([2.0], [2.0 + delta], [y], [math.sqrt(r)], [s], [c], [0.0], kinds=["real"])
    assert abs(L - ref) < 1e-14


def test_real_term_instantaneous_ar1():
    """Noiseless instantaneous samples of one real term: the textbook AR(1)
    likelihood, x_k | x_{k-1} ~ N(rho_k x_{k-1}, s^2 (1 - rho_k^2)),
    rho_k = exp(-c dt_k), x_1 ~ N(0, s^2)."""
    rng = np.random.default_rng(11)
    t = np.sort(rng.uniform(0, 5, 30))
    x = rng.normal(size=30)
    s, c = 0.9, 1.7
    ref = -0.5 * (math.log(2 * math.pi * s * s) + x[0] ** 2 / (s * s))
    for k in range(1, 30):
        rho = math.exp(-c * (t[k] - t[k - 1]))
        v = s * s * (1 - rho * rho)
        ref += -0.5 * (math.log(2 * math.pi * v) + (x[k] - rho * x[k - 1]) ** 2 / v)
    L = kalman.loglik(t, t, x, np.zeros(30), [s], [c], [1.0], kinds=["real"])
    assert abs(L - ref) < 1e-12 * abs(ref)


@pytest.mark.parametrize("kinds", [["real"], ["real", "sho"], ["sho", "real", "real"]])
def test_kalman_equals_dense_with_real_terms(kinds):
    M = len(kinds)
    b = W.random_small_batch(40 + M, B=2, n_lo=10, n_hi=35, M=M, J=3)
    for i in range(b.n_series):
        s = b.series(i)
        args = (s["ts"], s["te"], s["y"], s["yerr"], s["sigma"], s["omega0"], s["quality"], s["jitter"])
        Ld = dense.loglik(*args, kinds=kinds)
        Lk = kalman.loglik(*args, kinds=kinds)
        assert abs(Ld - Lk) <= 1e-11 * abs(Ld), (kinds, i, Ld, Lk)
        tt = np.linspace(s["ts"].min() - 0.05, s["te"].max() + 0.05, 11)
        md, vd, mt, vt = dense.posterior(*args, t_test=tt, kinds=kinds)
        _, mt2, vt2, md2, vd2 = kalman.smooth(*args, t_test=tt, kinds=kinds)
        k0 = float(np.sum(np.asarray(s["sigma"]) ** 2))
        assert np.max(np.abs(md - md2)) < 1e-11 * math.sqrt(k0) and np.max(np.abs(vd - vd2)) < 1e-11 * k0
        assert np.max(np.abs(mt - mt2)) < 1e-11 * math.sqrt(k0) and np.max(np.abs(vt - vt2)) < 1e-11 * k0


def test_dense_gradient_with_real_terms_matches_fd_of_kalman():
    kinds = ["sho", "real"]
    b = W.random_small_batch(51, B=1, n_lo=25, n_hi=25, M=2, J=2)
    s = b.series(0)
    args = (s["ts"], s["te"], s["y"], s["yerr"], s["sigma"], s["omega0"], s["quality"], s["jitter"])
    _, g = dense.loglik_grad(*args, kinds=kinds)
    gfd = kalman.loglik_grad_fd(*args, kinds=kinds)
    assert g[2 * 2 + 1] == 0.0 and gfd[2 * 2 + 1] == 0.0  # Q of the real term
    den = np.maximum(np.abs(gfd), 1e-3 * np.max(np.abs(gfd)))
    assert np.max(np.abs(g - gfd) / den) < 1e-6


def test_matern32_is_the_sho_term_at_half():
    """The Matern-3/2 kernel s^2 (1 + sqrt3 u/rho) exp(-sqrt3 u/rho), written
    out here and integrated over exposures by the same quadrature, equals the
    SHO term with Q = 1/2 and omega0 = sqrt3/rho."""
    s, rho = 0.7, 0.35
    rng = np.random.default_rng(2)
    ts = np.sort(rng.uniform(0, 2, 12))
    te = ts + rng.uniform(0, 0.2, 12)
    te[3] = ts[3]
    r3 = math.sqrt(3.0) / rho

    def matern(u):
        a = r3 * np.abs(u)
        return s * s * (1 + a) * np.exp(-a)

    Km = dense._pair_block(ts[:, None], te[:, None], ts[None, :], te[None, :], matern, r3)
    Ks = dense.covariance(ts, te, [s], [r3], [0.5])
    assert np.max(np.abs(Km - Ks)) < 1e-14 * s * s


# ---------------------------------------------------------------------------
# per-instrument amplitude and offset in the observation model (Sec. 2.2,
# the observation matrix scaled per instrument; Sec. 3.2.3, labels)
# ---------------------------------------------------------------------------

def _inst_case(seed, n=45, ni=3, J=3):
    b = W.random_small_batch(seed, B=1, n_lo=n, n_hi=n, M=2, J=J)
    s = b.series(0)
    rng = np.random.default_rng(seed + 100)
    inst = rng.integers(0, ni, len(s["ts"]))
    amp = rng.uniform(0.5, 1.8, ni)
    off = rng.normal(0.0, 0.5, ni)
    return s, inst, amp, off


def test_single_instrument_amplitude_scales_sigma():
    """One amplitude a for every measurement equals scaling each term's
    sigma by a (the kernel is quadratic in sigma); the offset c equals
    subtracting c from the data."""
    s, _, _, _ = _inst_case(61)
    n = len(s["ts"])
    a, c = 1.7, -0.35
    base = (s["ts"], s["te"])
    L1 = kalman.loglik(*base, s["y"], s["yerr"], s["sigma"], s["omega0"], s["quality"], s["jitter"],
                       amp=np.full(n, a), off=np.full(n, c))
    L2 = kalman.loglik(*base, s["y"] - c, s["yerr"], a * np.asarray(s["sigma"]), s["omega0"], s["quality"],
                       s["jitter"])
    assert abs(L1 - L2) < 1e-13 * abs(L2)


def test_amplitude_change_of_variables():
    """With no jitter, dividing each measurement (residual and noise) by its
    own a_n gives the amplitude-free problem, and the density changes by the
    Jacobian: L(y; a, c, yerr) = L((y - c)/a; 1, 0, yerr/a) - sum log a_n."""
    s, inst, amp, off = _inst_case(62)
    a_n, c_n = kalman.expand_instruments(inst, amp, off)
    args = (s["sigma"], s["omega0"], s["quality"], 0.0)
    L1 = kalman.loglik(s["ts"], s["te"], s["y"], s["yerr"], *args, amp=a_n, off=c_n)
    L2 = kalman.loglik(s["ts"], s["te"], (s["y"] - c_n) / a_n, s["yerr"] / a_n, *args)
    assert abs(L1 - (L2 - np.sum(np.log(a_n)))) < 1e-12 * abs(L1)
    # the dense side, same identity
    D1 = dense.loglik(s["ts"], s["te"], s["y"], s["yerr"], *args, amp=a_n, off=c_n)
    D2 = dense.loglik(s["ts"], s["te"], (s["y"] - c_n) / a_n, s["yerr"] / a_n, *args)
    assert abs(D1 - (D2 - np.sum(np.log(a_n)))) < 1e-12 * abs(D1)


def test_instruments_instantaneous_textbook_gp():
    """Instantaneous samples from several instruments: the Gaussian density
    of y with covariance A K A + diag(yerr^2 + jitter^2) and mean c, from
    scipy's multivariate normal."""
    import scipy.stats as ss
    rng = np.random.default_rng(63)
    t = np.sort(rng.uniform(0, 3, 30))
    inst = rng.integers(0, 3, 30)
    amp, off = np.array([1.0, 0.6, 1.4]), np.array([0.1, -0.3, 0.25])
    a_n, c_n = kalman.expand_instruments(inst, amp, off)
    y = rng.normal(size=30)
    yerr = rng.uniform(0.1, 0.3, 30)
    sig, w0, q, jit = [1.0, 0.5], [2.0, 9.0], [0.8, 0.4], 0.07
    K = sum(sho.kernel(t[:, None] - t[None, :], sig[m], w0[m], q[m]) for m in range(2))
    ref = ss.multivariate_normal(mean=c_n, cov=a_n[:, None] * K * a_n[None, :] + np.diag(yerr ** 2 + jit ** 2)).logpdf(y)
    L = kalman.loglik(t, t, y, yerr, sig, w0, q, jit, amp=a_n, off=c_n)
    assert abs(L - ref) < 1e-12 * abs(ref)


@pytest.mark.parametrize("seed", [64, 65])
def test_kalman_equals_dense_with_instruments(seed):
    s, inst, amp, off = _inst_case(seed)
    a_n, c_n = kalman.expand_instruments(inst, amp, off)
    args = (s["ts"], s["te"], s["y"], s["yerr"], s["sigma"], s["omega0"], s["quality"], s["jitter"])
    Ld = dense.loglik(*args, amp=a_n, off=c_n)
    Lk = kalman.loglik(*args, amp=a_n, off=c_n)
    assert abs(Ld - Lk) <= 1e-11 * abs(Ld)
    tt = np.linspace(s["ts"].min() - 0.05, s["te"].max() + 0.05, 9)
    md, vd, mt, vt = dense.posterior(*args, t_test=tt, amp=a_n, off=c_n)
    _, mt2, vt2, md2, vd2 = kalman.smooth(*args, t_test=tt, amp=a_n, off=c_n)
    k0 = float(np.sum(np.asarray(s["sigma"]) ** 2))
    assert np.max(np.abs(md - md2)) < 1e-11 * math.sqrt(k0) and np.max(np.abs(vd - vd2)) < 1e-11 * k0
    assert np.max(np.abs(mt - mt2)) < 1e-11 * math.sqrt(k0) and np.max(np.abs(vt - vt2)) < 1e-11 * k0


def test_dense_gradient_with_instruments_matches_fd_of_kalman():
    s, inst, amp, off = _inst_case(66, n=30)
    a_n, c_n = kalman.expand_instruments(inst, amp, off)
    args = (s["ts"], s["te"], s["y"], s["yerr"], s["sigma"], s["omega0"], s["quality"], s["jitter"])
    L, g = dense.loglik_grad(*args, instrument=inst, amp=amp, off=off)
    gt = kalman.loglik_grad_fd(*args, amp=a_n, off=c_n)
    gi = kalman.loglik_grad_inst_fd(*args, inst, amp, off)
    gfd = np.concatenate([gt, gi])
    assert g.shape == (3 * 2 + 1 + 6,)
    den = np.maximum(np.abs(gfd), 1e-3 * np.max(np.abs(gfd)))
    assert np.max(np.abs(g - gfd) / den) < 1e-6


def test_instrument_parameters_validated():
    s, inst, amp, off = _inst_case(67, n=10)
    a_n, c_n = kalman.expand_instruments(inst, amp, off)
    args = (s["ts"], s["te"], s["y"], s["yerr"], s["sigma"], s["omega0"], s["quality"], s["jitter"])
    for bad in (0.0, -1.0, np.nan, np.inf):
        a2 = a_n.copy()
        a2[3] = bad
        with pytest.raises(kalman.OracleError):
            kalman.loglik(*args, amp=a2, off=c_n)
    c2 = c_n.copy()
    c2[0] = np.nan
    with pytest.raises(kalman.OracleError):
        kalman.loglik(*args, amp=a_n, off=c2)


# ---------------------------------------------------------------------------
# high-precision dense oracle (closed-form exposure integrals, mpmath) and
# the square-root form of the sequential filter
# ---------------------------------------------------------------------------

def test_exact_covariance_matches_quadrature_and_appendix_a():
    """The closed-form window integrals (second antiderivative of the kernel)
    against the dense oracle's quadrature, and against Appendix A's
    exposure-averaged kernel for equal exposures."""
    from oracle import exact
    b = W.random_small_batch(81, B=1, n_lo=25, n_hi=25, M=2, J=3)
    s = b.series(0)
    te = s["te"].copy()
    te[4] = s["ts"][4]  # an instantaneous sample among exposures
    Ke = np.array(exact.covariance(s["ts"], te, s["sigma"], s["omega0"], s["quality"]).tolist(), dtype=float)
    Kd = dense.covariance(s["ts"], te, s["sigma"], s["omega0"], s["quality"])
    assert np.max(np.abs(Ke - Kd)) < 1e-13 * np.max(np.abs(Kd))
    sg, w0, q = 1.0, 2.0, 1.5
    eta = math.sqrt(1 - 1 / (4 * q * q))
    a, bb, c, d = sg * sg, sg * sg / (2 * eta * q), w0 / (2 * q), eta * w0
    delta = 0.7
    for lag in (0.0, 0.3, 2.5):
        ref = _celerite_integrated(a, bb, c, d, delta, lag)
        K = exact.covariance([0.0, lag], [delta, lag + delta], [sg], [w0], [q])
        assert abs(float(K[0, 1]) - ref) < 1e-14 * abs(ref) + 1e-16, (lag, float(K[0, 1]), ref)


def test_exact_loglik_matches_kalman_and_dense():
    from oracle import exact
    for seed in (82, 83):
        b = W.random_small_batch(seed, B=1, n_lo=30, n_hi=30, M=2, J=3)
        s = b.series(0)
        args = (s["ts"], s["te"], s["y"], s["yerr"], s["sigma"], s["omega0"], s["quality"], s["jitter"])
        Le = exact.loglik(*args)
        assert abs(Le - kalman.loglik(*args)) < 1e-12 * abs(Le)
        assert abs(Le - dense.loglik(*args)) < 1e-10 * abs(Le)
    g = exact.loglik_grad_fd(*args)
    gk = kalman.loglik_grad_fd(*args)
    den = np.maximum(np.abs(gk), 1e-3 * np.max(np.abs(gk)))
    assert np.max(np.abs(g - gk) / den) < 1e-6


@pytest.mark.parametrize("seed", [84, 85])
def test_sqrt_filter_equals_covariance_filter(seed):
    """The square-root form computes the same likelihood (with instruments'
    amplitudes and offsets, real terms and overlapping exposures)."""
    s, inst, amp, off = _inst_case(seed)
    a_n, c_n = kalman.expand_instruments(inst, amp, off)
    args = (s["ts"], s["te"], s["y"], s["yerr"], s["sigma"], s["omega0"], s["quality"], s["jitter"])
    for kinds in (None, ["sho", "real"]):
        L1 = kalman.loglik(*args, kinds=kinds, amp=a_n, off=c_n)
        L2 = kalman.loglik_sqrt(*args, kinds=kinds, amp=a_n, off=c_n)
        assert abs(L1 - L2) < 1e-13 * abs(L1), (kinds, L1, L2)


@pytest.mark.parametrize("instantaneous", [True, False])
def test_sqrt_and_exact_oracles_on_nearly_noise_free_data(instantaneous):
    """Dense sampling with measurement errors down to 1e-9 of the signal:
    the long-double filters (covariance and square-root form) against the
    high-precision dense likelihood."""
    import conditioning_cases as CC
    from oracle import exact
    for noise in (1e-5, 1e-9):
        ts, te, y, yerr, sig, w0, q = CC.smooth(31, 30, noise, 0.5, instantaneous)
        Le = exact.loglik(ts, te, y, yerr, sig, w0, q, 0.0, dps=80)
        Ls = kalman.loglik_sqrt(ts, te, y, yerr, sig, w0, q, 0.0)
        Lc = kalman.loglik(ts, te, y, yerr, sig, w0, q, 0.0)
        assert abs(Ls - Le) < 1e-12 * abs(Le), (noise, Le, Ls)
        assert abs(Lc - Le) < 1e-12 * abs(Le), (noise, Le, Lc)


def test_sqrt_and_covariance_oracles_across_long_gaps():
    """Series whose covariance factors meet subnormal squares in double
    precision (a fast term across one-day gaps): the long-double covariance
    and square-root filters agree with each other and with the dense GP."""
    import conditioning_cases as CC
    for seed in range(3):
        ts, te, y, yerr, sig, w0, q = CC.long_gaps(seed)
        Lc = kalman.loglik(ts, te, y, yerr, sig, w0, q, 0.0)
        Ls = kalman.loglik_sqrt(ts, te, y, yerr, sig, w0, q, 0.0)
        assert abs(Lc - Ls) < 1e-13 * abs(Lc), (seed, Lc, Ls)
    # the dense GP (quadrature and Cholesky) on a shorter draw of the same kind
    ts, te, y, yerr, sig, w0, q = CC.long_gaps(0, n=40)
    Lc = kalman.loglik(ts, te, y, yerr, sig, w0, q, 0.0)
    Ld = dense.loglik(ts, te, y, yerr, sig, w0, q, 0.0)
    assert abs(Lc - Ld) < 1e-10 * abs(Lc), (Lc, Ld)


def test_exact_posterior_matches_dense_and_kalman():
    """The high-precision posterior (data and test times) against the dense
    oracle's and the long-double smoother's, at ordinary noise."""
    from oracle import exact
    b = W.random_small_batch(86, B=1, n_lo=25, n_hi=25, M=2, J=3)
    s = b.series(0)
    args = (s["ts"], s["te"], s["y"], s["yerr"], s["sigma"], s["omega0"], s["quality"], s["jitter"])
    tt = np.linspace(s["ts"].min() - 0.05, s["te"].max() + 0.05, 9)
    md, vd = exact.posterior_data(*args)
    mt, vt = exact.posterior_test(*args[:7], tt, args[7])
    md2, vd2, mt2, vt2 = dense.posterior(*args, t_test=tt)
    _, mt3, vt3, md3, vd3 = kalman.smooth(*args, t_test=tt)
    k0 = float(np.sum(np.asarray(s["sigma"]) ** 2))
    for a, b_, c in ((md, md2, md3), (mt, mt2, mt3)):
        assert np.max(np.abs(a - b_)) < 1e-11 * math.sqrt(k0) and np.max(np.abs(a - c)) < 1e-12 * math.sqrt(k0)
    for a, b_, c in ((vd, vd2, vd3), (vt, vt2, vt3)):
        assert np.max(np.abs(a - b_)) < 1e-11 * k0 and np.max(np.abs(a - c)) < 1e-12 * k0
