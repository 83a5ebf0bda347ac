"""GPU parity over combinations of the optional model features: every term
count (1-4) with up to four overlapping exposures, each with real terms
mixed in, instrument amplitudes and offsets, or both, under two chunkings;
log-likelihood, gradient (sampled series, central differences of the
long-double oracle), smoother and square-root filter (sequential and split in
time) against the oracle.  These combinations select the extended kernels
(real terms, instrument tables) at every slot count, including those whose
per-event state spills to LDS (four open exposures).

Tolerances as in test_gpu_parity: log-likelihood 1e-9 relative, gradient
1e-6 (relative to max(|g_i|, 1e-3 max|g|)), smoothed moments 1e-9 of the
prior standard deviation / variance (times the amplitude for the data)."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import kalman

pytestmark = pytest.mark.gpu

SHAPES = [(1, 2), (2, 4), (3, 4), (4, 2), (4, 3)]
FEATURES = ["real", "inst", "real+inst"]


def _args(s):
    return (s["ts"], s["te"], s["y"], s["yerr"], s["sigma"], s["omega0"], s["quality"], s["jitter"])


def _grad_err(g, ref):
    den = np.maximum(np.abs(ref), 1e-3 * np.max(np.abs(ref)))
    return np.max(np.abs(g - ref) / den)


def _depth(b):
    return max(kalman.greedy_slots(b.series(i)["ts"], b.series(i)["te"])[1] for i in range(b.n_series))


def _case(M, J, feature, seed):
    # a short span, so that the exposures of J instruments overlap; the first
    # seed from `seed` on (step 1000) whose batch is J deep
    for k in range(50):
        b = W.random_small_batch(seed + 1000 * k, B=4, n_lo=20, n_hi=45, M=M, J=J, T=1.0)
        if _depth(b) == J:
            break
    assert _depth(b) == J
    kinds = None
    if "real" in feature:
        kinds = ["sho"] * M
        kinds[-1] = "real"
        if M > 2:
            kinds[0] = "real"
        for m, k in enumerate(kinds):
            if k == "real":
                b.quality[:, m] = -1.0  # not read for a real term
    lab = amp = off = None
    if "inst" in feature:
        rng = np.random.default_rng(seed + 7)
        ni = 3
        lab = rng.integers(0, ni, len(b.t_start)).astype(np.int32)
        amp = rng.uniform(0.6, 1.6, (b.n_series, ni))
        off = rng.normal(0.0, 0.3, (b.n_series, ni))
    return b, kinds, lab, amp, off


def _series_inst(b, lab, amp, off, i):
    if lab is None:
        return None, None, None
    lo, hi = int(b.offsets[i]), int(b.offsets[i + 1])
    a_n, c_n = kalman.expand_instruments(lab[lo:hi], amp[i], off[i])
    return lab[lo:hi], a_n, c_n


@pytest.mark.parametrize("feature", FEATURES)
@pytest.mark.parametrize("M,J", SHAPES)
def test_feature_matrix(lib, M, J, feature):
    seed = 900 + 10 * M + J + 100 * FEATURES.index(feature)
    b, kinds, lab, amp, off = _case(M, J, feature, seed)
    ni = 0 if lab is None else amp.shape[1]
    ref = []
    for i in range(b.n_series):
        _, a_n, c_n = _series_inst(b, lab, amp, off, i)
        ref.append(kalman.loglik(*_args(b.series(i)), kinds=kinds, amp=a_n, off=c_n))
    ref = np.array(ref)
    nt = 7
    tt = np.concatenate([np.linspace(b.series(i)["ts"].min() - 0.03, b.series(i)["te"].max() + 0.03, nt)
                         for i in range(b.n_series)])
    to = np.arange(b.n_series + 1, dtype=np.int64) * nt
    grads = []
    for opt in (dict(chunk_min=1, chunk_target=3), dict()):
        plan = lib.Plan(b.offsets, b.t_start, b.t_end, b.y, b.yerr, **opt)
        if kinds:
            plan.set_term_kinds(kinds)
        if lab is not None:
            plan.set_instruments(lab, ni)
            ll, g, st = plan.loglik_grad_inst(b.sigma, b.omega0, b.quality, b.jitter, amp, off, status=True)
        else:
            ll, g, st = plan.loglik_grad(b.sigma, b.omega0, b.quality, b.jitter, status=True)
        ll, g, st = ll.cpu().numpy(), g.cpu().numpy(), st.cpu().numpy()
        assert np.all(st == 0)
        assert plan.stats()["max_slots"] == J
        rel = np.max(np.abs(ll - ref) / np.abs(ref))
        print(M, J, feature, opt, plan.stats()["max_slots"], rel)
        assert rel < 1e-9
        # the square-root filter's kernel of the same feature set
        ls = plan.loglik_sqrt(b.sigma, b.omega0, b.quality, b.jitter, amp, off, check=True).cpu().numpy()
        assert np.max(np.abs(ls - ref) / np.abs(ref)) < 1e-9
        ls = plan.loglik_sqrt_split(b.sigma, b.omega0, b.quality, b.jitter, amp, off, check=True).cpu().numpy()
        assert np.max(np.abs(ls - ref) / np.abs(ref)) < 1e-9
        grads.append(g)
        o = plan.smooth(b.sigma, b.omega0, b.quality, b.jitter, to, tt, amp=amp, off=off)
        o = {k: v.cpu().numpy() for k, v in o.items() if v is not None}
        for i in (0, b.n_series - 1):
            s = b.series(i)
            _, a_n, c_n = _series_inst(b, lab, amp, off, i)
            _, mt, vt, md, vd = kalman.smooth(*_args(s), t_test=tt[to[i]:to[i + 1]], kinds=kinds, amp=a_n, off=c_n)
            k0 = float(np.sum(np.asarray(s["sigma"]) ** 2))
            lo, hi = int(b.offsets[i]), int(b.offsets[i + 1])
            am = 1.0 if amp is None else float(np.max(amp[i]))
            errs = (np.max(np.abs(o["mean_data"][lo:hi] - md)) / (am * math.sqrt(k0)),
                    np.max(np.abs(o["var_data"][lo:hi] - vd)) / (am * am * k0),
                    np.max(np.abs(o["mean_test"][to[i]:to[i + 1]] - mt)) / math.sqrt(k0),
                    np.max(np.abs(o["var_test"][to[i]:to[i + 1]] - vt)) / k0)
            assert max(errs) < 1e-9, (opt, i, errs)
    assert _grad_err(grads[0], grads[1]) < 1e-9
    i = int(np.argmax([b.offsets[k + 1] - b.offsets[k] for k in range(b.n_series)]))
    s = b.series(i)
    li, a_n, c_n = _series_inst(b, lab, amp, off, i)
    gfd = kalman.loglik_grad_fd(*_args(s), kinds=kinds, amp=a_n, off=c_n)
    if lab is not None:
        gfd = np.concatenate([gfd, kalman.loglik_grad_inst_fd(*_args(s), li, amp[i], off[i], kinds=kinds)])
    g = grads[1][i]
    if kinds:
        real_q = [2 * M + m for m, k in enumerate(kinds) if k == "real"]
        assert np.all(g[real_q] == 0.0)
    e = _grad_err(g, gfd)
    print("gradient", i, e)
    assert e < 1e-6, (g, gfd)
