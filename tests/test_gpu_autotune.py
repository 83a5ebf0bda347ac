"""The autotuner (gp_ssm_autotune): every candidate it can pick is a plan
whose results match the oracle, and its choice is one of the candidates,
stored in and read back from its cache, and overridden by
GP_SSM_TARGET_CHUNKS.

Tolerances as in test_gpu_parity: log-likelihood 1e-9 relative, gradient
1e-6 (relative to max(|g_i|, 1e-3 max|g|))."""
import os

import numpy as np
import pytest

import workloads as W
from oracle import kalman

pytestmark = pytest.mark.gpu


def _args(s):
    return (s["ts"], s["te"], s["y"], s["yerr"], s["sigma"], s["omega0"], s["quality"], s["jitter"])


def _grad_err(g, ref):
    den = np.maximum(np.abs(ref), 1e-3 * np.max(np.abs(ref)))
    return np.max(np.abs(g - ref) / den)


def test_every_candidate_matches_oracle(lib):
    """The 1024-series gradient batch under every candidate target chunk count
    (from 16 to 512 chunks per series): sampled series against the oracle."""
    b = W.grad_1024()
    sample = [0, 700]
    ref = {i: kalman.loglik(*_args(b.series(i))) for i in sample}
    gref = kalman.loglik_grad_fd(*_args(b.series(0)))
    cands = lib.autotune_candidates()
    assert len(cands) >= 4
    seen = set()
    for tc in cands:
        plan = lib.Plan(b.offsets, b.t_start, b.t_end, b.y, b.yerr, target_chunks=tc)
        st = plan.stats()
        seen.add(st["n_chunks"])
        ll, g = plan.loglik_grad(b.sigma, b.omega0, b.quality, b.jitter)
        ll, g = ll.cpu().numpy(), g.cpu().numpy()
        assert np.all(np.isfinite(ll)) and np.all(np.isfinite(g))
        rels = [abs(ll[i] - ref[i]) / abs(ref[i]) for i in sample]
        ge = _grad_err(g[0], gref)
        print(tc, st["n_chunks"], st["max_chunk_len"], rels, ge)
        assert max(rels) < 1e-9 and ge < 1e-6
        del plan
    assert len(seen) >= 3  # the candidates make different plans


def test_autotune_choice_cache_and_override(lib, tmp_path):
    b = W.random_small_batch(71, B=64, n_lo=100, n_hi=800, M=2, J=2, T=30.0)
    cache = str(tmp_path / "tune.txt")
    inputs = (b.offsets, b.t_start, b.t_end, b.y, b.yerr, b.sigma, b.omega0, b.quality, b.jitter)
    opt, ms = lib.autotune(*inputs, grad=True, cache=cache)
    print(opt, ms)
    assert opt["target_chunks"] in lib.autotune_candidates() and ms > 0
    lines = open(cache).read().splitlines()
    assert len(lines) == 1 and lines[0].split()[1] == str(opt["target_chunks"])
    opt2, ms2 = lib.autotune(*inputs, grad=True, cache=cache)
    assert opt2 == opt and abs(ms2 - ms) < 1e-5 * ms
    assert len(open(cache).read().splitlines()) == 1
    os.environ["GP_SSM_TARGET_CHUNKS"] = "12345"
    try:
        opt3, _ = lib.autotune(*inputs, grad=False, cache=False)
    finally:
        del os.environ["GP_SSM_TARGET_CHUNKS"]
    assert opt3["target_chunks"] == 12345
    plan = lib.Plan(b.offsets, b.t_start, b.t_end, b.y, b.yerr, **opt)
    ll = plan.loglik(b.sigma, b.omega0, b.quality, b.jitter).cpu().numpy()
    for i in (0, 63):
        ref = kalman.loglik(*_args(b.series(i)))
        assert abs(ll[i] - ref) / abs(ref) < 1e-9
