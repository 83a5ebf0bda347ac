"""ORACLE -- test infrastructure only.

The dense integrated Gaussian process, i.e. the plain definition that the
augmented state-space method reaches exactly, only faster.

* Covariance between two exposure-averaged measurements (Sec. 3.1, integrated
  covariance; read with delta_1 and delta_2 the two exposure lengths):
      K_ij = 1/(d_i d_j) int_{t_i^s}^{t_i^e} int_{t_j^s}^{t_j^e} k(t - t') dt' dt
  reduced to one dimension, int k(|u|) l_ij(u) du, where the overlap length
  l_ij(u) of window i with window j shifted by u is a trapezoid.  Each linear
  piece of the trapezoid, split at u = 0 (where k(|u|) has a kink), is
  integrated by Gauss-Legendre quadrature on sub-pieces short compared with
  the kernel's fastest rate.  A zero-length exposure is an instantaneous
  sample (one integral, or the kernel itself when both are instantaneous).
* Log-likelihood: Cholesky of K + diag(yerr^2 + jitter^2) (Sec. 2.1 /
  Sec. 2.4, the Gaussian marginal likelihood).
* Posterior at the data and at test times (Sec. 2.1, GP conditioning), with
  K_* the kernel averaged over each exposure and K_** = k(0).
* Gradient: 1/2 tr((alpha alpha^T - K_y^-1) dK_y/dtheta) (standard Gaussian
  marginal-likelihood gradient; not in the paper), dK/dtheta from the same
  quadrature of the kernel's analytic derivative.
* Per-instrument amplitude and offset (Sec. 2.2, the observation matrix
  scaled per instrument; Sec. 3.2.3, instrument labels): measurement n reads
  a_n times its exposure average plus c_n, so K_y = A K A + diag(noise) with
  A = diag(a_n), and the residual is y - c.  The gradient in a_i uses
  dK_y/da_i = E_i K A + A K E_i (E_i the indicator of instrument i's rows);
  the one in c_i is the sum of alpha over instrument i's rows.
"""
from __future__ import annotations

import numpy as np
from numpy.polynomial.legendre import leggauss
from scipy.linalg import cho_factor, cho_solve

from . import sho

_NG = 16
_XG, _WG = leggauss(_NG)
_LOG2PI = np.log(2 * np.pi)


def _is_real(kinds, m):
    return kinds is not None and kinds[m] in ("real", 1)


def _rate(omega0, quality, kinds=None):
    omega0 = np.atleast_1d(omega0)
    quality = np.atleast_1d(quality)
    return float(max(omega0[m] * (1.0 if _is_real(kinds, m) else 1 + 1 / quality[m]) for m in range(len(omega0))))


def _kern_sum(u, sigma, omega0, quality, which=None, dtheta=None, kinds=None):
    """sum_m k_m(|u|), or with which=(m, name) the derivative of term m with
    respect to sigma, omega0 or Q.  kinds: per term 'sho' (default) or 'real'
    (sigma^2 exp(-omega0 |u|), Appendix A with b = d = 0; Q unused)."""
    sigma = np.atleast_1d(sigma)
    omega0 = np.atleast_1d(omega0)
    quality = np.atleast_1d(quality)
    if which is None:
        out = 0.0
        for m in range(len(sigma)):
            if _is_real(kinds, m):
                out = out + sho.real_kernel(u, sigma[m], omega0[m])
            else:
                out = out + sho.kernel(u, sigma[m], omega0[m], quality[m])
        return out
    m, name = which
    if _is_real(kinds, m):
        if name == "quality":
            return np.zeros_like(np.asarray(u, dtype=np.float64))
        return sho.real_kernel_grad(u, sigma[m], omega0[m])[{"sigma": 0, "omega0": 1}[name]]
    if name == "sigma":
        return 2.0 / sigma[m] * sho.kernel(u, sigma[m], omega0[m], quality[m])
    g = sho.kernel_grad(u, sigma[m], omega0[m], quality[m])
    return g[{"omega0": 1, "quality": 2}[name]]


def _integrate_linear(lo, hi, p, q, kfun, rate):
    """int_lo^hi k(|u|) (p + q u) du for arrays of intervals, split at 0 and
    subdivided so each sub-piece has rate * length <= 0.5."""
    lo = np.asarray(lo, dtype=np.float64)
    hi = np.asarray(hi, dtype=np.float64)
    z = np.clip(0.0, lo, hi)
    total = np.zeros_like(lo)
    for a, b in ((lo, z), (z, hi)):
        length = b - a
        nsub = max(1, int(np.ceil(np.max(length, initial=0.0) * rate / 0.5)))
        for s in range(nsub):
            a_s = a + length * (s / nsub)
            b_s = a + length * ((s + 1) / nsub)
            half = 0.5 * (b_s - a_s)
            mid = 0.5 * (b_s + a_s)
            u = mid[..., None] + half[..., None] * _XG
            w = half[..., None] * _WG
            total = total + np.sum(w * kfun(u) * (p[..., None] + q[..., None] * u), axis=-1)
    return total


def _pair_block(tsi, tei, tsj, tej, kfun, rate):
    """Integrated covariance for arrays of pairs (broadcast shapes)."""
    di = tei - tsi
    dj = tej - tsj
    shape = np.broadcast(tsi, tsj).shape
    tsi, tei, tsj, tej, di, dj = (np.broadcast_to(v, shape).astype(np.float64) for v in (tsi, tei, tsj, tej, di, dj))
    out = np.zeros(shape)
    zi = di <= 0
    zj = dj <= 0
    # both instantaneous
    both = zi & zj
    if np.any(both):
        out[both] = kfun(tsi[both] - tsj[both])
    # i instantaneous, j integrated: (1/dj) int_{t_i - te_j}^{t_i - ts_j} k(|u|) du
    oi = zi & ~zj
    if np.any(oi):
        lo = tsi[oi] - tej[oi]
        hi = tsi[oi] - tsj[oi]
        out[oi] = _integrate_linear(lo, hi, np.ones_like(lo), np.zeros_like(lo), kfun, rate) / dj[oi]
    oj = zj & ~zi
    if np.any(oj):
        lo = tsj[oj] - tei[oj]
        hi = tsj[oj] - tsi[oj]
        out[oj] = _integrate_linear(lo, hi, np.ones_like(lo), np.zeros_like(lo), kfun, rate) / di[oj]
    gen = ~zi & ~zj
    if np.any(gen):
        a, b, c, d = tsi[gen], tei[gen], tsj[gen], tej[gen]
        corners = np.sort(np.stack([a - d, a - c, b - d, b - c]), axis=0)
        c1, c2, c3, c4 = corners
        # overlap length: rises on [c1,c2] (u - c1), flat (c2 - c1) on [c2,c3], falls (c4 - u) on [c3,c4]
        one = np.ones_like(c1)
        zero = np.zeros_like(c1)
        v = _integrate_linear(c1, c2, -c1, one, kfun, rate)
        v = v + _integrate_linear(c2, c3, c2 - c1, zero, kfun, rate)
        v = v + _integrate_linear(c3, c4, c4, -one, kfun, rate)
        out[gen] = v / (di[gen] * dj[gen])
    return out


def covariance(ts, te, sigma, omega0, quality, which=None, block=256, kinds=None):
    """Dense integrated covariance matrix (or its derivative, see
    ``_kern_sum``)."""
    ts = np.asarray(ts, dtype=np.float64)
    te = np.asarray(te, dtype=np.float64)
    n = len(ts)
    rate = _rate(omega0, quality, kinds)

    def kfun(u):
        return _kern_sum(u, sigma, omega0, quality, which, kinds=kinds)

    K = np.zeros((n, n))
    for r0 in range(0, n, block):
        r1 = min(n, r0 + block)
        K[r0:r1, :] = _pair_block(ts[r0:r1, None], te[r0:r1, None], ts[None, :], te[None, :], kfun, rate)
    return 0.5 * (K + K.T)


def cross_covariance(t_test, ts, te, sigma, omega0, quality, block=256, kinds=None):
    """K_*: covariance between the latent f(t*) and each exposure average."""
    t_test = np.asarray(t_test, dtype=np.float64)
    ts = np.asarray(ts, dtype=np.float64)
    te = np.asarray(te, dtype=np.float64)
    rate = _rate(omega0, quality, kinds)

    def kfun(u):
        return _kern_sum(u, sigma, omega0, quality, kinds=kinds)

    out = np.zeros((len(ts), len(t_test)))
    for r0 in range(0, len(ts), block):
        r1 = min(len(ts), r0 + block)
        tq = t_test[None, :]
        out[r0:r1] = _pair_block(ts[r0:r1, None], te[r0:r1, None], tq, tq, kfun, rate)
    return out


def _scaled(K, y, amp, off):
    """(A K A, y - c) for per-measurement amplitudes and offsets (None: 1, 0)."""
    y = np.asarray(y, dtype=np.float64)
    if amp is not None:
        a = np.asarray(amp, dtype=np.float64)
        K = a[:, None] * K * a[None, :]
    if off is not None:
        y = y - np.asarray(off, dtype=np.float64)
    return K, y


def loglik(ts, te, y, yerr, sigma, omega0, quality, jitter=0.0, K=None, kinds=None, amp=None, off=None):
    if K is None:
        K = covariance(ts, te, sigma, omega0, quality, kinds=kinds)
    K, y = _scaled(K, y, amp, off)
    Ky = K + np.diag(np.asarray(yerr) ** 2 + jitter ** 2)
    cf = cho_factor(Ky, lower=True)
    alpha = cho_solve(cf, y)
    return float(-0.5 * y @ alpha - np.sum(np.log(np.diag(cf[0]))) - 0.5 * len(y) * _LOG2PI)


def posterior_terms(ts, te, y, yerr, sigma, omega0, quality, jitter=0.0, t_test=None):
    """Component-wise latent posterior at t_test (Appendix C, component-wise
    predictive means and variances): for each term m the cross-covariance
    K_{m,*} of that term alone with the data, mean K_{m,*}^T K_y^-1 y and
    variance sigma_m^2 - K_{m,*}^T K_y^-1 K_{m,*}.  Returns (mean, var), each
    [n_test, M], and the per-term cross-covariances [M][n, n_test]."""
    sigma, omega0, quality = (np.atleast_1d(np.asarray(a, dtype=np.float64)) for a in (sigma, omega0, quality))
    K = covariance(ts, te, sigma, omega0, quality)
    Ky = K + np.diag(np.asarray(yerr) ** 2 + jitter ** 2)
    cf = cho_factor(Ky, lower=True)
    alpha = cho_solve(cf, np.asarray(y, dtype=np.float64))
    M = len(sigma)
    mean = np.zeros((len(t_test), M))
    var = np.zeros((len(t_test), M))
    Ks = []
    for m in range(M):
        Km = cross_covariance(t_test, ts, te, sigma[m:m + 1], omega0[m:m + 1], quality[m:m + 1])
        mean[:, m] = Km.T @ alpha
        var[:, m] = sigma[m] ** 2 - np.sum(Km * cho_solve(cf, Km), axis=0)
        Ks.append(Km)
    return mean, var, Ks


def posterior(ts, te, y, yerr, sigma, omega0, quality, jitter=0.0, t_test=None, kinds=None, amp=None, off=None):
    """(mean_data, var_data, mean_test, var_test): posterior of the
    noise-free measured quantity a_n * (exposure average) + c_n at the data
    and latent posterior at t_test."""
    K, yr = _scaled(covariance(ts, te, sigma, omega0, quality, kinds=kinds), y, amp, off)
    Ky = K + np.diag(np.asarray(yerr) ** 2 + jitter ** 2)
    cf = cho_factor(Ky, lower=True)
    alpha = cho_solve(cf, yr)
    mean_d = K @ alpha + (0.0 if off is None else np.asarray(off, dtype=np.float64))
    var_d = np.diag(K) - np.sum(K * cho_solve(cf, K), axis=0)
    if t_test is None:
        return mean_d, var_d, None, None
    Ks = cross_covariance(t_test, ts, te, sigma, omega0, quality, kinds=kinds)
    if amp is not None:
        Ks = np.asarray(amp, dtype=np.float64)[:, None] * Ks
    mean_t = Ks.T @ alpha
    k0 = float(np.sum(np.atleast_1d(sigma) ** 2))
    var_t = k0 - np.sum(Ks * cho_solve(cf, Ks), axis=0)
    return mean_d, var_d, mean_t, var_t


def loglik_grad(ts, te, y, yerr, sigma, omega0, quality, jitter=0.0, kinds=None, instrument=None, amp=None,
                off=None):
    """Analytic gradient ordered (d sigma_1..M, d omega0_1..M, d Q_1..M,
    d jitter), together with the log-likelihood.  With instrument labels
    (int per measurement) and per-instrument amp and off (length I), the
    gradient continues with (d amp_0..I-1, d off_0..I-1)."""
    sigma = np.atleast_1d(np.asarray(sigma, dtype=np.float64))
    omega0 = np.atleast_1d(np.asarray(omega0, dtype=np.float64))
    quality = np.atleast_1d(np.asarray(quality, dtype=np.float64))
    M = len(sigma)
    K0 = covariance(ts, te, sigma, omega0, quality, kinds=kinds)
    a_n = c_n = None
    if instrument is not None:
        inst = np.asarray(instrument, dtype=np.int64)
        a_n = np.asarray(amp, dtype=np.float64)[inst]
        c_n = np.asarray(off, dtype=np.float64)[inst]
    K, y = _scaled(K0, y, a_n, c_n)
    Ky = K + np.diag(np.asarray(yerr) ** 2 + jitter ** 2)
    cf = cho_factor(Ky, lower=True)
    alpha = cho_solve(cf, y)
    Kinv = cho_solve(cf, np.eye(len(y)))
    W = np.outer(alpha, alpha) - Kinv
    L = float(-0.5 * y @ alpha - np.sum(np.log(np.diag(cf[0]))) - 0.5 * len(y) * _LOG2PI)
    ni = 0 if instrument is None else len(amp)
    g = np.zeros(3 * M + 1 + 2 * ni)
    for k, name in enumerate(("sigma", "omega0", "quality")):
        for m in range(M):
            dK = covariance(ts, te, sigma, omega0, quality, which=(m, name), kinds=kinds)
            g[k * M + m] = 0.5 * np.sum(W * _scaled(dK, y, a_n, None)[0])
    g[3 * M] = 0.5 * np.trace(W) * 2 * jitter
    for i in range(ni):
        E = (inst == i).astype(np.float64)
        KA = K0 * a_n[None, :]
        dK = E[:, None] * KA + KA.T * E[None, :]
        g[3 * M + 1 + i] = 0.5 * np.sum(W * dK)
        g[3 * M + 1 + ni + i] = float(np.sum(alpha[inst == i]))
    return L, g
