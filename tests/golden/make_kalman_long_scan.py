"""Writes kalman_long_scan.json: the sequential oracle's log-likelihood
(oracle/kalman.c, long double) and its central-difference gradient
(relative steps 1e-6) for two series long enough that the GPU's
time-parallel scan, cut at every quiet point, needs its second level
(more than 64 x 64 chunks):

* "c5_prefix": 32000 exposures from the generator of the 1e7-exposure
  workload (workloads.long_1e7) at the same density (4 instruments, three
  terms, up to four overlapping exposures);
* "m4": 12000 exposures of a random series with four terms and two
  instruments (workloads.random_small_batch).

Calls only workloads and oracle/.  Takes a few minutes:

    python tests/golden/make_kalman_long_scan.py
"""
import json
import multiprocessing as mp
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

CASES = {
    "c5_prefix": ("long_1e7", dict(n=32000, T=3652.5 * 32000 / 1e7)),
    "m4": ("random_small_batch", dict(seed=404, B=1, n_lo=12000, n_hi=12000, M=4, J=2, T=3000.0)),
}


def make(name):
    import workloads as W
    fn, kw = CASES[name]
    return getattr(W, fn)(**kw)


def one(name):
    from oracle import kalman
    s = make(name).series(0)
    a = (s["ts"], s["te"], s["y"], s["yerr"], s["sigma"], s["omega0"], s["quality"], s["jitter"])
    L = kalman.loglik(*a)
    g = kalman.loglik_grad_fd(*a)
    print(name, "done", flush=True)
    return {"name": name, "generator": CASES[name][0], "kwargs": CASES[name][1], "loglik": float(L),
            "grad_fd": [float(v) for v in g]}


if __name__ == "__main__":
    with mp.Pool(len(CASES)) as pool:
        rows = pool.map(one, list(CASES))
    with open(os.path.join(HERE, "kalman_long_scan.json"), "w") as fh:
        json.dump({"source": "oracle/kalman.c loglik and loglik_grad_fd", "cases": rows}, fh, indent=1)
