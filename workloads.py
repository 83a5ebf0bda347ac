"""Seeded synthetic inputs shared by the tests, the smoke check and the
benchmark.

This module holds no arithmetic of the method: it only places exposure
windows, draws hyperparameters and measurement errors, and makes surrogate
measurements.  The surrogate signal is a sum of random-phase sinusoids per
SHO term, with frequencies scattered around the term's omega0 and amplitude
sigma, averaged analytically over each exposure window; noise of variance
yerr^2 + jitter^2 is added.  It has the scale and time structure of a draw
from the process but is not one (the benchmarks and parity tests do not
depend on the data being an exact draw).

Time unit: days.  Exposure durations given in minutes or seconds are
converted (1 min = 1/1440 d).

Workloads (names used by the tests and the benchmark):

  small_single   one instrument, 180 s exposures with no dead time, an SHO
                 with a ~300 s timescale, errors 0.3 (the paper's
                 single-instrument validation scenario, synthetic)
  small_multi    two instruments with 55 s and 180 +- 30 s exposures that
                 frequently overlap (the paper's two-instrument validation
                 scenario, synthetic)
  single_1k      1 series, N = 1000 non-overlapping exposures on [0, 100] d,
                 durations U(5, 30) min, one SHO term sigma = 1,
                 omega0 = 2 pi/10 d^-1, Q = 1/sqrt 2, errors 0.1
  long_100k      1 series, N = 1e5 over 365 d, 3 instruments, durations
                 U(1, 20) min, terms (1, 2 pi/0.2, 1/sqrt 2) +
                 (0.5, 2 pi 1440/5, 30), lognormal errors (median 0.2,
                 log-sd 0.5), 1e4 evenly spaced test times
  batch_4096     4096 series, N_b log-uniform in [1e3, 5e4], 2 instruments,
                 2 terms each with omega0 log-uniform [0.1, 1000], Q
                 log-uniform [0.5, 50], sigma log-uniform [0.1, 2]
  grad_1024      1024 series of N = 1e4, 3 instruments, 3 terms (ranges as
                 batch_4096) and jitter 0.05
  long_1e7       1 series, N = 1e7 over 3652.5 d, 4 instruments, durations
                 U(20, 100) s, terms of long_100k plus (2, 2 pi/30, 1/sqrt 2)

Exposures of one instrument are placed by the spacing construction: for n
durations d_i on [0, T], draw u = sort(U(0, T - sum d, n)) and set
t_start_i = u_i + sum_{k<i} d_k; this is the uniform distribution over
non-overlapping placements.  Instruments are placed independently and
merged (sorted by start time), so at most as many exposures overlap as there
are instruments.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

MIN = 1.0 / 1440.0
SEC = MIN / 60.0


@dataclass
class Batch:
    """A batch of series in the flat layout the library takes."""
    offsets: np.ndarray          # int64 [B+1]
    t_start: np.ndarray          # float64 [N]
    t_end: np.ndarray            # float64 [N]
    y: np.ndarray                # float64 [N]
    yerr: np.ndarray             # float64 [N]
    sigma: np.ndarray            # float64 [B, M]
    omega0: np.ndarray           # float64 [B, M]
    quality: np.ndarray          # float64 [B, M]
    jitter: np.ndarray           # float64 [B]
    name: str = ""
    t_test: np.ndarray | None = None         # float64 [T] (all series)
    test_offsets: np.ndarray | None = None   # int64 [B+1]
    meta: dict = field(default_factory=dict)

    @property
    def n_series(self):
        return len(self.offsets) - 1

    @property
    def n_terms(self):
        return self.sigma.shape[1]

    def series(self, b):
        a, e = int(self.offsets[b]), int(self.offsets[b + 1])
        return dict(ts=self.t_start[a:e], te=self.t_end[a:e], y=self.y[a:e], yerr=self.yerr[a:e],
                    sigma=self.sigma[b], omega0=self.omega0[b], quality=self.quality[b],
                    jitter=float(self.jitter[b]))

    def subset(self, idx):
        idx = list(idx)
        parts = [self.series(b) for b in idx]
        lens = [len(p["ts"]) for p in parts]
        off = np.zeros(len(idx) + 1, dtype=np.int64)
        off[1:] = np.cumsum(lens)
        return Batch(off, np.concatenate([p["ts"] for p in parts]), np.concatenate([p["te"] for p in parts]),
                     np.concatenate([p["y"] for p in parts]), np.concatenate([p["yerr"] for p in parts]),
                     self.sigma[idx].copy(), self.omega0[idx].copy(), self.quality[idx].copy(),
                     self.jitter[idx].copy(), self.name + "[subset]")


def place_slot(rng, T, durations, t0=0.0):
    """Uniform non-overlapping placement of exposures of the given durations
    on [t0, t0 + T]."""
    durations = np.asarray(durations, dtype=np.float64)
    free = T - durations.sum()
    if free < 0:
        raise ValueError("exposures do not fit in the interval")
    u = np.sort(rng.uniform(0.0, free, len(durations)))
    ts = t0 + u + np.concatenate([[0.0], np.cumsum(durations)[:-1]])
    return ts, ts + durations


def surrogate_y(rng, ts, te, yerr, jitter, sigma, omega0, quality, n_waves=8):
    """Sum of random-phase sinusoids per term, averaged over each window,
    plus white noise."""
    ts = np.asarray(ts)
    te = np.asarray(te)
    d = te - ts
    f = np.zeros(len(ts))
    for s, w, q in zip(np.atleast_1d(sigma), np.atleast_1d(omega0), np.atleast_1d(quality)):
        nu = w * np.exp(rng.normal(0.0, 0.5 / q + 0.05, n_waves))
        ph = rng.uniform(0, 2 * np.pi, n_waves)
        amp = s * math.sqrt(2.0 / n_waves)
        for k in range(n_waves):
            inst = np.cos(nu[k] * ts + ph[k])
            with np.errstate(divide="ignore", invalid="ignore"):
                avg = (np.sin(nu[k] * te + ph[k]) - np.sin(nu[k] * ts + ph[k])) / (nu[k] * d)
            f += amp * np.where(d > 0, avg, inst)
    return f + rng.normal(0.0, 1.0, len(ts)) * np.sqrt(np.asarray(yerr) ** 2 + jitter ** 2)


def _series(rng, T, slot_counts, dur_lo, dur_hi, sigma, omega0, quality, jitter, yerr_fn, n_waves=8):
    tss, tes = [], []
    for n in slot_counts:
        d = rng.uniform(dur_lo, dur_hi, n)
        ts, te = place_slot(rng, T, d)
        tss.append(ts)
        tes.append(te)
    ts = np.concatenate(tss)
    te = np.concatenate(tes)
    order = np.argsort(ts, kind="stable")
    ts, te = ts[order], te[order]
    yerr = yerr_fn(len(ts))
    y = surrogate_y(rng, ts, te, yerr, jitter, sigma, omega0, quality, n_waves)
    return ts, te, y, yerr


def _pack(name, parts, sigma, omega0, quality, jitter, t_test=None, test_offsets=None, meta=None):
    lens = [len(p[0]) for p in parts]
    off = np.zeros(len(parts) + 1, dtype=np.int64)
    off[1:] = np.cumsum(lens)
    cat = [np.concatenate([p[i] for p in parts]) for i in range(4)]
    return Batch(off, cat[0], cat[1], cat[2], cat[3], np.asarray(sigma, dtype=np.float64),
                 np.asarray(omega0, dtype=np.float64), np.asarray(quality, dtype=np.float64),
                 np.asarray(jitter, dtype=np.float64), name, t_test, test_offsets, meta or {})


def _loguniform(rng, lo, hi, size):
    return np.exp(rng.uniform(math.log(lo), math.log(hi), size))


def lognormal_errors(rng, median=0.2, log_sd=0.5):
    return lambda n: median * np.exp(log_sd * rng.normal(size=n))


# ---------------------------------------------------------------------------
# named workloads
# ---------------------------------------------------------------------------

def single_1k(seed=1, n=1000):
    rng = np.random.default_rng(seed)
    sig, w0, q = [1.0], [2 * np.pi / 10], [1 / np.sqrt(2)]
    part = _series(rng, 100.0, [n], 5 * MIN, 30 * MIN, sig, w0, q, 0.0, lambda k: np.full(k, 0.1))
    return _pack("single_1k", [part], [sig], [w0], [q], [0.0])


def long_100k(seed=2, n=100_000, n_test=10_000, T=365.0):
    rng = np.random.default_rng(seed)
    sig = [1.0, 0.5]
    w0 = [2 * np.pi / 0.2, 2 * np.pi * 1440 / 5]
    q = [1 / np.sqrt(2), 30.0]
    counts = [n // 3 + (1 if i < n % 3 else 0) for i in range(3)]
    part = _series(rng, T, counts, 1 * MIN, 20 * MIN, sig, w0, q, 0.0, lognormal_errors(rng))
    t_test = np.linspace(0.0, T, n_test)
    return _pack("long_100k", [part], [sig], [w0], [q], [0.0], t_test,
                 np.array([0, n_test], dtype=np.int64))


def _random_terms(rng, B, M):
    w0 = _loguniform(rng, 0.1, 1000.0, (B, M))
    q = _loguniform(rng, 0.5, 50.0, (B, M))
    sig = _loguniform(rng, 0.1, 2.0, (B, M))
    return sig, w0, q


def batch_4096(seed=3, B=4096, n_lo=1000, n_hi=50_000, T=365.0, n_waves=2):
    rng = np.random.default_rng(seed)
    sig, w0, q = _random_terms(rng, B, 2)
    nb = np.round(_loguniform(rng, n_lo, n_hi, B)).astype(np.int64)
    parts = []
    err = lognormal_errors(rng)
    for b in range(B):
        counts = [int(nb[b]) // 2, int(nb[b]) - int(nb[b]) // 2]
        parts.append(_series(rng, T, counts, 1 * MIN, 20 * MIN, sig[b], w0[b], q[b], 0.0, err, n_waves))
    return _pack("batch_4096", parts, sig, w0, q, np.zeros(B))


def grad_1024(seed=4, B=1024, n=10_000, T=365.0, jitter=0.05):
    rng = np.random.default_rng(seed)
    sig, w0, q = _random_terms(rng, B, 3)
    parts = []
    err = lognormal_errors(rng)
    counts = [n // 3 + (1 if i < n % 3 else 0) for i in range(3)]
    for b in range(B):
        parts.append(_series(rng, T, counts, 1 * MIN, 20 * MIN, sig[b], w0[b], q[b], jitter, err))
    return _pack("grad_1024", parts, sig, w0, q, np.full(B, jitter))


def long_1e7(seed=5, n=10_000_000, T=3652.5, n_waves=4):
    rng = np.random.default_rng(seed)
    sig = [1.0, 0.5, 2.0]
    w0 = [2 * np.pi / 0.2, 2 * np.pi * 1440 / 5, 2 * np.pi / 30]
    q = [1 / np.sqrt(2), 30.0, 1 / np.sqrt(2)]
    counts = [n // 4 + (1 if i < n % 4 else 0) for i in range(4)]
    part = _series(rng, T, counts, 20 * SEC, 100 * SEC, sig, w0, q, 0.0, lognormal_errors(rng), n_waves)
    return _pack("long_1e7", [part], [sig], [w0], [q], [0.0])


def small_single(seed=11, n=40):
    """Single instrument, 180 s exposures back to back (no dead time)."""
    rng = np.random.default_rng(seed)
    d = 180 * SEC
    gaps = np.where(rng.uniform(size=n) < 0.7, 0.0, rng.uniform(0, 600 * SEC, n))
    ts = np.cumsum(np.concatenate([[0.0], (d + gaps)[:-1]]))
    te = ts + d
    sig, w0, q = [1.0], [2 * np.pi / (300 * SEC)], [1.0]
    yerr = np.full(n, 0.3)
    y = surrogate_y(rng, ts, te, yerr, 0.0, sig, w0, q)
    return _pack("small_single", [(ts, te, y, yerr)], [sig], [w0], [q], [0.0],
                 np.linspace(-0.002, te[-1] + 0.002, 97), np.array([0, 97], dtype=np.int64))


def small_multi(seed=12, n1=30, n2=12):
    """Two instruments: 55 s exposures and 180 +- 30 s exposures that
    frequently overlap."""
    rng = np.random.default_rng(seed)
    T = 0.06
    ts1, te1 = place_slot(rng, T, np.full(n1, 55 * SEC))
    ts2, te2 = place_slot(rng, T, np.clip(rng.normal(180, 30, n2), 60, 300) * SEC)
    ts = np.concatenate([ts1, ts2])
    te = np.concatenate([te1, te2])
    o = np.argsort(ts, kind="stable")
    ts, te = ts[o], te[o]
    sig, w0, q = [1.0, 0.3], [2 * np.pi / (300 * SEC), 2 * np.pi / (0.05)], [3.0, 1 / np.sqrt(2)]
    yerr = rng.uniform(0.1, 0.3, len(ts))
    y = surrogate_y(rng, ts, te, yerr, 0.0, sig, w0, q)
    return _pack("small_multi", [(ts, te, y, yerr)], [sig], [w0], [q], [0.0],
                 np.linspace(-0.003, T + 0.003, 101), np.array([0, 101], dtype=np.int64))


def random_small_batch(seed, B=8, n_lo=3, n_hi=60, M=2, J=3, T=2.0, jitter=True, instant_frac=0.1,
                       tie_frac=0.1):
    """Small random batches for parity tests: uneven lengths, overlaps up to
    J instruments, some zero-length exposures and exact time ties."""
    rng = np.random.default_rng(seed)
    sig, w0, q = _loguniform(rng, 0.2, 2.0, (B, M)), _loguniform(rng, 0.3, 300.0, (B, M)), \
        _loguniform(rng, 0.3, 40.0, (B, M))
    jit = rng.uniform(0.0, 0.1, B) if jitter else np.zeros(B)
    parts = []
    for b in range(B):
        n = int(rng.integers(n_lo, n_hi + 1))
        counts = np.bincount(rng.integers(0, J, n), minlength=J)
        tss, tes = [], []
        for c in counts:
            if c == 0:
                continue
            d = rng.uniform(0.001, 0.05, c)
            d[rng.uniform(size=c) < instant_frac] = 0.0
            ts, te = place_slot(rng, T, d)
            # back-to-back ties inside the instrument
            tie = rng.uniform(size=c) < tie_frac
            for i in range(1, c):
                if tie[i] and d[i - 1] > 0 and d[i] > 0:
                    shift = ts[i] - te[i - 1]
                    ts[i:] -= shift
                    te[i:] -= shift
            tss.append(ts)
            tes.append(te)
        ts = np.concatenate(tss)
        te = np.concatenate(tes)
        o = np.argsort(ts, kind="stable")
        ts, te = ts[o], te[o]
        yerr = rng.uniform(0.05, 0.3, len(ts))
        y = surrogate_y(rng, ts, te, yerr, jit[b], sig[b], w0[b], q[b])
        parts.append((ts, te, y, yerr))
    return _pack("random_small", parts, sig, w0, q, jit)


WORKLOADS = {
    "single_1k": single_1k,
    "long_100k": long_100k,
    "batch_4096": batch_4096,
    "grad_1024": grad_1024,
    "long_1e7": long_1e7,
    "small_single": small_single,
    "small_multi": small_multi,
}
