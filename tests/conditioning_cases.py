"""Nearly noise-free, densely sampled series for the conditioning tests (CPU
pins of the square-root and high-precision oracles, GPU parity): a smooth
process observed many times per correlation time with measurement errors
1e-5 ... 1e-9 of its amplitude, so that each measurement is almost
predicted by the previous ones (innovation variance close to R).  The data
are a draw from the dense integrated GP itself (the oracle's high-precision
covariance, rounded to double), so that the likelihood is typical."""
import numpy as np

from oracle import exact


def _draw(rng, ts, te, sigma, omega0, quality, yerr):
    K = np.array(exact.covariance(ts, te, sigma, omega0, quality, dps=50).tolist(), dtype=np.float64)
    w, V = np.linalg.eigh(K)
    return V @ (np.sqrt(np.clip(w, 0.0, None)) * rng.normal(size=len(ts))) + yerr * rng.normal(size=len(ts))


def smooth(seed, n, noise, omega0, instantaneous, T=2.0, max_exposure=0.005):
    """One SHO term (sigma 1, Q 1/sqrt 2), n samples on [0, T]."""
    rng = np.random.default_rng(seed)
    ts = np.sort(rng.uniform(0.0, T, n))
    te = ts.copy() if instantaneous else ts + rng.uniform(0.0, max_exposure, n)
    sig, w0, q = np.array([1.0]), np.array([omega0]), np.array([1.0 / np.sqrt(2.0)])
    yerr = np.full(n, noise)
    y = _draw(rng, ts, te, sig, w0, q, yerr)
    return ts, te, y, yerr, sig, w0, q


def two_instruments(seed, n, noise, T=5.0):
    """Two SHO terms, two instruments whose exposures (0.02-0.1 d) overlap."""
    rng = np.random.default_rng(seed)
    ts, te = [], []
    for k in (n // 2, n - n // 2):
        d = rng.uniform(0.02, 0.1, k)
        u = np.sort(rng.uniform(0.0, T - d.sum(), k))
        s0 = u + np.concatenate([[0.0], np.cumsum(d)[:-1]])
        ts.append(s0)
        te.append(s0 + d)
    ts, te = np.concatenate(ts), np.concatenate(te)
    o = np.argsort(ts, kind="stable")
    ts, te = ts[o], te[o]
    sig, w0, q = np.array([1.0, 0.3]), np.array([0.3, 2.0]), np.array([2.0, 0.7])
    yerr = np.full(n, noise * np.sqrt(np.sum(sig ** 2)))
    y = _draw(rng, ts, te, sig, w0, q, yerr)
    return ts, te, y, yerr, sig, w0, q


def long_gaps(seed, n=120):
    """A fast term (omega0 860 / d, Q 1.22) beside a slow one, with gaps of
    about one day between 1-20 minute exposures: over such a gap the fast
    term's transition is e^(-350) or so, so that factors of the covariance
    carry entries whose squares are subnormal in double precision."""
    rng = np.random.default_rng(seed)
    gaps = rng.choice([0.5, 0.98, 1.0, 1.01, 1.02, 1.03, 1.04, 1.05, 1.2], n) + rng.uniform(0.0, 0.01, n)
    ts = np.cumsum(gaps)
    te = ts + rng.uniform(1.0 / 1440, 20.0 / 1440, n)
    yerr = rng.uniform(0.15, 0.25, n)
    y = rng.normal(0.0, 0.5, n)
    return ts, te, y, yerr, np.array([0.37, 0.15]), np.array([860.0, 0.95]), np.array([1.22, 1.7])
