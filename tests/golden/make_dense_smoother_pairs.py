"""Writes dense_smoother_pairs.json: the dense oracle's posterior
(oracle/dense.py: GP conditioning with the integrated covariance from
quadrature) at the data and at test times, for short series in which two
exposures start almost together:

* "pair3ms": 60 exposures of two instruments with one pair of starts 3 ms
  apart (the construction of the oracle's own smoother-accuracy pin);
* "long_100k_w<k>": 301-exposure windows of the 1e5-exposure smoother
  workload (workloads.long_100k) centred on each start pair closer than
  0.02 s, each taken as a series of its own.

The test times of each case: 40 evenly spaced over the window and 20 in the
0.1 day (or the window's span) before the pair.  Calls only workloads and
oracle/.  Takes a few minutes:

    python tests/golden/make_dense_smoother_pairs.py
"""
import json
import multiprocessing as mp
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402


def pair3ms():
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
    yerr = np.full(len(ts), 0.2)
    y = rng.normal(size=len(ts)) * 0.5
    return dict(name="pair3ms", ts=ts, te=te, y=y, yerr=yerr, sigma=[1.0, 0.5],
                omega0=[2 * np.pi / 0.2, 2 * np.pi * 1440 / 5], quality=[1 / np.sqrt(2), 30.0], jitter=0.0)


def windows():
    b = W.long_100k()
    s = b.series(0)
    ts = s["ts"]
    at = np.flatnonzero(np.diff(ts) * 86400.0 < 0.02) + 1
    out = []
    for k, i in enumerate(at):
        lo, hi = max(0, i - 150), min(len(ts), i + 151)
        out.append(dict(name=f"long_100k_w{k}", ts=ts[lo:hi], te=s["te"][lo:hi], y=s["y"][lo:hi],
                        yerr=s["yerr"][lo:hi], sigma=list(s["sigma"]), omega0=list(s["omega0"]),
                        quality=list(s["quality"]), jitter=float(s["jitter"]), pair_index=int(i - lo)))
    return out


def test_times(c):
    ts, te = c["ts"], c["te"]
    p = c.get("pair_index", int(np.argmin(np.diff(ts))) + 1)
    tp = ts[p]
    before = np.linspace(max(ts[0], tp - 0.1), tp, 20, endpoint=False)
    return np.sort(np.concatenate([np.linspace(ts[0] - 0.01, te[-1] + 0.01, 40), before]))


def one(c):
    from oracle import dense
    tt = test_times(c)
    md, vd, mt, vt = dense.posterior(c["ts"], c["te"], c["y"], c["yerr"], c["sigma"], c["omega0"], c["quality"],
                                     c["jitter"], t_test=tt)
    print(c["name"], "done", flush=True)
    row = {k: (v.tolist() if isinstance(v, np.ndarray) else v) for k, v in c.items()}
    row.update(t_test=tt.tolist(), mean_data=md.tolist(), var_data=vd.tolist(), mean_test=mt.tolist(),
               var_test=vt.tolist())
    return row


if __name__ == "__main__":
    cases = [pair3ms()] + windows()
    with mp.Pool(len(cases)) as pool:
        rows = pool.map(one, cases)
    with open(os.path.join(HERE, "dense_smoother_pairs.json"), "w") as fh:
        json.dump({"source": "oracle/dense.py posterior", "cases": rows}, fh)
