"""ORACLE -- test infrastructure only.

The SHO kernel and its state-space representation as the paper writes them
(Appendix B), for pinning the oracle's other parts.

* ``kernel``       the SHO covariance k(Delta) (Appendix B, SHO kernel), in a
                   form that is entire in eta^2 so it stays finite at Q = 1/2;
                   ``kernel_grad`` gives its analytic derivatives.
* ``psd``          its power spectral density (Appendix B, PSD).
* ``ssm``          F, L, Qc and Pinf of the SHO (Appendix B; Qc and the
                   stationary covariance from the Lyapunov equation).
* ``closed_forms`` the printed closed forms of the transition matrix, the
                   process noise, the integrated transition matrix and the
                   augmented noise blocks (Appendix B), evaluated in mpmath at
                   high precision.  They are printed for Q > 1/2; Q < 1/2 is
                   taken by analytic continuation in eta (every expression is
                   even in eta) and Q = 1/2 as the limit, read off at
                   Q = 1/2 + 10^-(dps/2).
"""
from __future__ import annotations

import mpmath as mp
import numpy as np


# ---------------------------------------------------------------------------
# kernel and PSD
# ---------------------------------------------------------------------------

def _ecs(a, w):
    """exp(-a) cos(sqrt w), exp(-a) sin(sqrt w)/sqrt w and exp(-a) times the
    w-derivative of sin(sqrt w)/sqrt w, for real a >= 0 and real w (w < 0 is
    the hyperbolic, overdamped branch).  Entire in w; series for |w| < 1e-2,
    exponentials combined with exp(-a) otherwise so nothing overflows."""
    a = np.asarray(a, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    a, w = np.broadcast_arrays(a, w)
    ea = np.exp(-a)
    small = np.abs(w) < 1e-2
    ws = np.where(small, w, 0.0)
    c = np.zeros_like(ws)
    s = np.zeros_like(ws)
    ds = np.zeros_like(ws)
    tc = np.ones_like(ws)
    tsr = np.ones_like(ws)
    for n in range(9):
        c += tc
        s += tsr
        # d/dw of (-w)^n/(2n+1)!  = -n (-w)^(n-1)/(2n+1)!
        if n >= 1:
            ds += -n * tsr_prev_over_w(ws, n)
        tc = tc * (-ws) / ((2 * n + 1) * (2 * n + 2))
        tsr = tsr * (-ws) / ((2 * n + 2) * (2 * n + 3))
    ser = (ea * c, ea * s, ea * ds)
    wl = np.where(small, 1.0, w)
    pos = wl > 0
    r = np.sqrt(np.abs(wl))
    # oscillatory branch
    ec_p = ea * np.cos(r)
    es_p = ea * np.sin(r) / r
    # hyperbolic branch: exp(-a) cosh r = (exp(r - a) + exp(-r - a)) / 2
    ep = np.exp(np.minimum(r - a, 700.0))
    em = np.exp(-r - a)
    ec_n = 0.5 * (ep + em)
    es_n = 0.5 * (ep - em) / r
    ec = np.where(pos, ec_p, ec_n)
    es = np.where(pos, es_p, es_n)
    eds = (ec - es) / (2 * wl)
    return (np.where(small, ser[0], ec), np.where(small, ser[1], es), np.where(small, ser[2], eds))


def tsr_prev_over_w(ws, n):
    """(-w)^(n-1)/(2n+1)! (helper of the series of d/dw sin(sqrt w)/sqrt w)."""
    return (-ws) ** (n - 1) / float(np.prod(np.arange(1, 2 * n + 2, dtype=np.float64)))


def _aw(tau, omega0, quality):
    t = np.abs(np.asarray(tau, dtype=np.float64))
    x = omega0 * t
    a = x / (2 * quality)
    w = (1 - 1 / (4 * quality * quality)) * x * x
    return x, a, w


def kernel(tau, sigma, omega0, quality):
    """SHO covariance at lag |tau| (Appendix B, SHO kernel):
    sigma^2 exp(-w0 t / 2Q) [cos(eta w0 t) + sin(eta w0 t) / (2 eta Q)],
    with the Q <= 1/2 branches as the same entire function of eta^2:
    sigma^2 exp(-a) [cos r + a sin(r)/r],  a = w0 t/2Q,
    r^2 = w = (1 - 1/4Q^2)(w0 t)^2."""
    x, a, w = _aw(tau, omega0, quality)
    ec, es, _ = _ecs(a, w)
    return sigma * sigma * (ec + a * es)


def kernel_grad(tau, sigma, omega0, quality):
    """Partial derivatives of ``kernel`` with respect to (sigma, omega0, Q),
    by the chain rule through a and w:
      dk/da = sigma^2 exp(-a) [s - c - a s],
      dk/dw = sigma^2 exp(-a) [-s/2 + a ds/dw],
      da/domega0 = a/omega0, dw/domega0 = 2 w/omega0,
      da/dQ = -a/Q, dw/dQ = (w0 t)^2 / (2 Q^3)."""
    x, a, w = _aw(tau, omega0, quality)
    ec, es, eds = _ecs(a, w)
    k = sigma * sigma * (ec + a * es)
    dka = sigma * sigma * (es - ec - a * es)
    dkw = sigma * sigma * (-0.5 * es + a * eds)
    d_sigma = 2 * k / sigma
    d_omega0 = dka * a / omega0 + dkw * 2 * w / omega0
    d_quality = -dka * a / quality + dkw * x * x / (2 * quality ** 3)
    return d_sigma, d_omega0, d_quality


def real_kernel(tau, sigma, c):
    """Real (exponential) term, the celerite term of Appendix A with
    b = d = 0: sigma^2 exp(-c |tau|)."""
    return sigma * sigma * np.exp(-c * np.abs(tau))


def real_kernel_grad(tau, sigma, c):
    """Partial derivatives of ``real_kernel`` with respect to (sigma, c)."""
    k = real_kernel(tau, sigma, c)
    return 2 * k / sigma, -np.abs(tau) * k


def psd(omega, sigma, omega0, quality):
    """Power spectral density of the SHO (Appendix B, PSD) with
    S0 = sigma^2 / (omega0 Q)."""
    S0 = sigma * sigma / (omega0 * quality)
    return 2 * S0 * omega0 ** 4 / ((omega ** 2 - omega0 ** 2) ** 2 + omega0 ** 2 * omega ** 2 / quality ** 2)


def ssm(sigma, omega0, quality):
    """F, L, Qc and Pinf of the SHO state-space model (Appendix B)."""
    F = np.array([[0.0, 1.0], [-omega0 ** 2, -omega0 / quality]])
    L = np.array([[0.0], [1.0]])
    Qc = 2 * omega0 ** 3 * sigma ** 2 / quality
    Pinf = sigma ** 2 * np.diag([1.0, omega0 ** 2])
    return F, L, Qc, Pinf


# ---------------------------------------------------------------------------
# Appendix B closed forms in mpmath
# ---------------------------------------------------------------------------

def closed_forms(sigma, omega0, quality, dt, dps=60):
    """Appendix B closed forms for one SHO term over a step dt.

    Returns a dict of numpy float arrays:
      Phi   (2x2)  transition matrix (SHO transition)
      Qk    (2x2)  process noise (SHO process noise, Q > 1/2 form)
      Phibar(2x2)  integrated transition matrix (SHO integrated transition)
      q12   (2,)   first column of the augmented cross block (augmented noise
                   cross block)
      q22   ()     the augmented integrated-integrated element
    """
    with mp.workdps(dps):
        s = mp.mpf(sigma)
        w0 = mp.mpf(omega0)
        Q = mp.mpf(quality)
        D = mp.mpf(dt)
        if Q == mp.mpf(1) / 2:
            Q = Q + mp.mpf(10) ** (-(dps // 2))
        eta2 = 1 - 1 / (4 * Q * Q)
        eta = mp.sqrt(eta2) if eta2 > 0 else mp.mpc(0, 1) * mp.sqrt(-eta2)
        A = 1 / (2 * eta * Q)
        tau = eta * w0 * D
        ex = mp.exp(-w0 * D / (2 * Q))
        exx = mp.exp(-w0 * D / Q)
        sn = mp.sin(tau)
        cs = mp.cos(tau)
        # transition
        Phi = [[ex * (cs + A * sn), ex * sn / (eta * w0)], [-ex * w0 * sn / eta, ex * (cs - A * sn)]]
        # process noise
        Qaa = mp.exp(w0 * D / Q) - 1 - A * mp.sin(2 * tau) - sn * sn / (2 * eta2 * Q * Q)
        Qab = w0 * sn * sn / (eta2 * Q)
        Qbb = w0 * w0 * (mp.exp(w0 * D / Q) - 1 + A * mp.sin(2 * tau) - sn * sn / (2 * eta2 * Q * Q))
        Qk = [[s * s * exx * Qaa, s * s * exx * Qab], [s * s * exx * Qab, s * s * exx * Qbb]]
        # integrated transition: e^{at}/(a^2+b^2) [[Ic + A Is, B Is],[C Is, Ic - A Is]] from 0 to dt
        a = -w0 / (2 * Q)
        b = eta * w0
        B = 1 / (eta * w0)
        C = -w0 / eta

        def prim(t):
            tt = eta * w0 * t
            Is = a * mp.sin(tt) - b * mp.cos(tt)
            Ic = a * mp.cos(tt) + b * mp.sin(tt)
            f = mp.exp(a * t) / (a * a + b * b)
            return [[f * (Ic + A * Is), f * B * Is], [f * C * Is, f * (Ic - A * Is)]]

        p1 = prim(D)
        p0 = prim(0)
        Phibar = [[p1[i][j] - p0[i][j] for j in range(2)] for i in range(2)]
        # augmented noise blocks
        q12 = [s * s / (Q * w0) * (ex * (cs + A * sn) - 1) ** 2,
               s * s * (A * ex * (4 * sn - ex * mp.sin(2 * tau)) - 2 * A * A * exx * sn * sn + exx - 1)]
        q22 = s * s / (4 * Q * Q * w0 * w0) * (
            8 * Q * w0 * D + 4 * Q * Q - 12 + A * A * exx * (mp.cos(2 * tau) - 16 * Q ** 4)
            + 16 * ex * (cs + (1 - 2 * Q * Q) * A * sn)
            + exx * ((1 - 3 * A * A) / A * mp.sin(2 * tau) - 3 * mp.cos(2 * tau)))

        def re(v):
            return float(mp.re(v))

        return {
            "Phi": np.array([[re(v) for v in row] for row in Phi]),
            "Qk": np.array([[re(v) for v in row] for row in Qk]),
            "Phibar": np.array([[re(v) for v in row] for row in Phibar]),
            "q12": np.array([re(v) for v in q12]),
            "q22": re(q22),
        }
