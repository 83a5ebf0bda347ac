"""ORACLE -- test infrastructure only.

The dense integrated Gaussian process in high-precision arithmetic (mpmath),
with the exposure integrals of the SHO kernel in closed form: the reference
for data whose measurement noise is so small that double precision, and the
covariance form of the long-double filter, lose digits.

* Kernel (Appendix B): for each SHO term, k(tau) = sigma^2 e^{-alpha tau}
  [cos(eta w0 tau) + sin(eta w0 tau) / (2 eta Q)] for tau >= 0, alpha =
  w0/(2Q), eta = sqrt(1 - 1/(4Q^2)) (imaginary for Q < 1/2; the expression
  is real either way), written as c_+ e^{l_+ tau} + c_- e^{l_- tau}.
* Exposure-averaged covariance (Sec. 3.1, integrated covariance): with F the
  even second antiderivative of k(|u|) (F(0) = F'(0) = 0),
      int_{a1}^{b1} int_{a2}^{b2} k(t - t') dt' dt
          = F(b1 - a2) - F(b1 - b2) - F(a1 - a2) + F(a1 - b2),
  divided by both exposure lengths; one instantaneous sample uses the first
  antiderivative, two use k itself.
* Log-likelihood (Sec. 2.4): Cholesky of K + diag(yerr^2 + jitter^2); its
  gradient by central differences at high precision.
* Posterior (Sec. 2.1, GP conditioning): at the data, K K_y^-1 y and
  diag(K - K K_y^-1 K); at test times, with the cross-covariances of the
  latent f(t*) and the exposure averages (the first antiderivative) and
  k(0).
Q = 1/2 exactly (eta = 0) is not supported.
"""
from __future__ import annotations

import mpmath as mp
import numpy as np


def _terms(sigma, omega0, quality):
    out = []
    for s, w, q in zip(sigma, omega0, quality):
        s, w, q = mp.mpf(s), mp.mpf(w), mp.mpf(q)
        eta = mp.sqrt(mp.mpc(1) - 1 / (4 * q * q))
        a = w / (2 * q)
        for sg in (1, -1):
            lam = -a + sg * 1j * eta * w
            c = s * s / 2 * (1 - sg * 1j / (2 * eta * q))
            out.append((c, lam))
    return out


def _k(terms, u):
    u = abs(u)
    return mp.re(sum(c * mp.exp(l * u) for c, l in terms))


def _k1(terms, u):
    """First antiderivative of k(|w|) from 0 (odd)."""
    au = abs(u)
    v = mp.re(sum(c * (mp.exp(l * au) - 1) / l for c, l in terms))
    return v if u >= 0 else -v


def _k2(terms, u):
    """Second antiderivative of k(|w|) from 0 (even)."""
    au = abs(u)
    return mp.re(sum(c * (mp.exp(l * au) - 1 - l * au) / (l * l) for c, l in terms))


def covariance(ts, te, sigma, omega0, quality, dps=40):
    """Exposure-averaged covariance matrix (mpmath matrix)."""
    with mp.workdps(dps):
        T = _terms(list(sigma) if np.ndim(sigma) else [sigma], list(omega0) if np.ndim(omega0) else [omega0],
                   list(quality) if np.ndim(quality) else [quality])
        a = [mp.mpf(x) for x in ts]
        b = [mp.mpf(x) for x in te]
        n = len(a)
        K = mp.matrix(n, n)
        for i in range(n):
            for j in range(i, n):
                di, dj = b[i] - a[i], b[j] - a[j]
                if di == 0 and dj == 0:
                    v = _k(T, a[i] - a[j])
                elif di == 0:
                    v = (_k1(T, a[i] - a[j]) - _k1(T, a[i] - b[j])) / dj
                elif dj == 0:
                    v = (_k1(T, a[j] - a[i]) - _k1(T, a[j] - b[i])) / di
                else:
                    v = (_k2(T, b[i] - a[j]) - _k2(T, b[i] - b[j]) - _k2(T, a[i] - a[j]) + _k2(T, a[i] - b[j])) / (
                        di * dj)
                K[i, j] = K[j, i] = v
        return K


def loglik(ts, te, y, yerr, sigma, omega0, quality, jitter=0.0, dps=40):
    with mp.workdps(dps):
        return float(_loglik_mp(ts, te, y, yerr, np.atleast_1d(sigma), np.atleast_1d(omega0), np.atleast_1d(quality),
                                jitter, dps))


def loglik_grad_fd(ts, te, y, yerr, sigma, omega0, quality, jitter=0.0, rel_step=1e-8, dps=60):
    """Central differences of loglik in (sigma_1..M, omega0_1..M, Q_1..M,
    jitter) with relative steps rel_step (absolute at a zero jitter, one
    sided there), in high precision, so the steps can be small."""
    with mp.workdps(dps):
        th = [mp.mpf(v) for v in list(np.atleast_1d(sigma)) + list(np.atleast_1d(omega0)) +
              list(np.atleast_1d(quality)) + [jitter]]
        M = len(np.atleast_1d(sigma))

        def L(t):
            return _loglik_mp(ts, te, y, yerr, t[:M], t[M:2 * M], t[2 * M:3 * M], t[3 * M], dps)

        g = []
        for i in range(len(th)):
            h = mp.mpf(rel_step) * (abs(th[i]) if th[i] != 0 else 1)
            tp = list(th)
            tp[i] += h
            if i == 3 * M and th[i] == 0:
                g.append(float((L(tp) - L(th)) / h))
                continue
            tm = list(th)
            tm[i] -= h
            g.append(float((L(tp) - L(tm)) / (2 * h)))
        return np.array(g)


def _loglik_mp(ts, te, y, yerr, sigma, omega0, quality, jitter, dps):
    with mp.workdps(dps):
        K = covariance(ts, te, sigma, omega0, quality, dps)
        n = len(y)
        for i in range(n):
            K[i, i] += mp.mpf(yerr[i]) ** 2 + mp.mpf(jitter) ** 2
        L = mp.cholesky(K)
        z = _forward(L, mp.matrix([mp.mpf(v) for v in y]))
        quad = sum(z[i] ** 2 for i in range(n))
        logdet = 2 * sum(mp.log(L[i, i]) for i in range(n))
        return -(quad + logdet + n * mp.log(2 * mp.pi)) / 2


def posterior_data(ts, te, y, yerr, sigma, omega0, quality, jitter=0.0, dps=40):
    """Posterior mean and variance of the noise-free exposure averages at the
    data (Sec. 2.1 GP conditioning): K K_y^-1 y and diag(K - K K_y^-1 K)."""
    with mp.workdps(dps):
        K = covariance(ts, te, sigma, omega0, quality, dps)
        n = len(y)
        Ky = K.copy()
        for i in range(n):
            Ky[i, i] += mp.mpf(yerr[i]) ** 2 + mp.mpf(jitter) ** 2
        L = mp.cholesky(Ky)
        z = _forward(L, mp.matrix([mp.mpf(v) for v in y]))
        alpha = _backward(L, z)
        mean = np.array([float(sum(K[i, k] * alpha[k] for k in range(n))) for i in range(n)])
        var = np.zeros(n)
        for i in range(n):
            w = _forward(L, mp.matrix([K[k, i] for k in range(n)]))
            var[i] = float(K[i, i] - sum(w[k] ** 2 for k in range(n)))
        return mean, var


def posterior_test(ts, te, y, yerr, sigma, omega0, quality, t_test, jitter=0.0, dps=40):
    """Posterior mean and variance of the latent f at the test times (Sec. 2.1
    GP conditioning, with the exposure-averaged cross-covariances)."""
    with mp.workdps(dps):
        T = _terms(list(np.atleast_1d(sigma)), list(np.atleast_1d(omega0)), list(np.atleast_1d(quality)))
        K = covariance(ts, te, sigma, omega0, quality, dps)
        n = len(y)
        for i in range(n):
            K[i, i] += mp.mpf(yerr[i]) ** 2 + mp.mpf(jitter) ** 2
        L = mp.cholesky(K)
        alpha = _backward(L, _forward(L, mp.matrix([mp.mpf(v) for v in y])))
        k0 = _k(T, mp.mpf(0))
        mean, var = np.zeros(len(t_test)), np.zeros(len(t_test))
        for q, tq in enumerate(t_test):
            tq = mp.mpf(tq)
            ks = mp.matrix(n, 1)
            for i in range(n):
                a, b = mp.mpf(ts[i]), mp.mpf(te[i])
                ks[i] = _k(T, tq - a) if b == a else (_k1(T, tq - a) - _k1(T, tq - b)) / (b - a)
            mean[q] = float(sum(ks[i] * alpha[i] for i in range(n)))
            w = _forward(L, ks)
            var[q] = float(k0 - sum(w[i] ** 2 for i in range(n)))
        return mean, var


def _backward(L, z):
    n = L.rows
    x = mp.matrix(n, 1)
    for i in reversed(range(n)):
        s = z[i]
        for k in range(i + 1, n):
            s -= L[k, i] * x[k]
        x[i] = s / L[i, i]
    return x


def _forward(L, b):
    n = L.rows
    z = mp.matrix(n, 1)
    for i in range(n):
        s = b[i]
        for k in range(i):
            s -= L[i, k] * z[k]
        z[i] = s / L[i, i]
    return z
