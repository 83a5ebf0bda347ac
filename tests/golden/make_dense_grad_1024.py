"""Writes dense_grad_1024.json: the dense oracle's log-likelihood and analytic
gradient (oracle/dense.py: quadrature of the integrated kernel, Cholesky, the
standard Gaussian marginal-likelihood gradient) on the first 500 exposures of
eight series of the 1024-series gradient batch (workloads.grad_1024), for the
GPU test that compares the adjoint gradient with it.  Calls only workloads
and oracle/.  Takes about an hour on eight cores:

    python tests/golden/make_dense_grad_1024.py
"""
import json
import multiprocessing as mp
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

SERIES = [0, 129, 258, 387, 516, 645, 774, 903]
N = 500


def one(i):
    import workloads as W
    from oracle import dense
    b = W.grad_1024()
    s = b.series(i)
    L, g = dense.loglik_grad(s["ts"][:N], s["te"][:N], s["y"][:N], s["yerr"][:N], s["sigma"], s["omega0"],
                             s["quality"], s["jitter"])
    print("series", i, "done", flush=True)
    return {"series": i, "n": N, "loglik": float(L), "grad": [float(v) for v in g]}


if __name__ == "__main__":
    with mp.Pool(min(len(SERIES), os.cpu_count() or 1)) as pool:
        rows = pool.map(one, SERIES)
    out = {"source": "oracle/dense.py loglik_grad on workloads.grad_1024(), first 500 exposures of each series",
           "rows": rows}
    with open(os.path.join(HERE, "dense_grad_1024.json"), "w") as fh:
        json.dump(out, fh, indent=1)
