"""GPU parity of the square-root (Cholesky-factor) filter
(gp_ssm_plan_loglik_sqrt, 16 lanes per series): against the oracle's
covariance-form and square-root filters on random batches at every term and
slot count, with real terms and per-instrument amplitudes and offsets, on
nearly noise-free series against the high-precision dense oracle, on the
per-series status contract, and against the batched time-parallel path on
the full 1024-series gradient workload.

Tolerances: 1e-9 relative to the oracle (as for the batched path); 1e-10
relative between the two GPU paths on the full workload, whose likelihoods
differ only in rounding (both FP64, different accumulation order)."""
import json
import os

import numpy as np
import pytest

import conditioning_cases as CC
import workloads as W
from oracle import exact, kalman

pytestmark = pytest.mark.gpu

TOL = 1e-9


def _args(s):
    return (s["ts"], s["te"], s["y"], s["yerr"], s["sigma"], s["omega0"], s["quality"], s["jitter"])


def _plan(lib, b, **opt):
    return lib.Plan(b.offsets, b.t_start, b.t_end, b.y, b.yerr, **opt)


@pytest.mark.parametrize("M,J,T", [(1, 1, 2.0), (1, 3, 2.0), (2, 2, 2.0), (2, 3, 2.0), (3, 3, 2.0), (3, 4, 0.4),
                                   (4, 2, 2.0), (4, 4, 0.4)])
def test_sqrt_matches_oracle(lib, M, J, T):
    # the first seed whose batch reaches overlap depth J (the kernel for J slots)
    for seed in range(900 + 100 * M + 10 * J, 1000 + 100 * M + 10 * J):
        b = W.random_small_batch(seed, B=6, n_lo=5, n_hi=70 if T > 1 else 40, M=M, J=J, T=T)
        plan = _plan(lib, b)
        if plan.stats()["max_slots"] == J:
            break
    assert plan.stats()["max_slots"] == J
    ll, st = plan.loglik_sqrt(b.sigma, b.omega0, b.quality, b.jitter, status=True)
    ll = ll.cpu().numpy()
    assert np.all(st.cpu().numpy() == 0)
    ref = np.array([kalman.loglik(*_args(b.series(i))) for i in range(b.n_series)])
    ref_sqrt = np.array([kalman.loglik_sqrt(*_args(b.series(i))) for i in range(b.n_series)])
    batched = plan.loglik(b.sigma, b.omega0, b.quality, b.jitter).cpu().numpy()
    rel = np.abs(ll - ref) / np.abs(ref)
    rel_sqrt = np.abs(ll - ref_sqrt) / np.abs(ref_sqrt)
    print(M, J, plan.stats()["max_slots"], rel.max(), rel_sqrt.max(), np.max(np.abs(ll - batched) / np.abs(ref)))
    assert rel.max() < TOL and rel_sqrt.max() < TOL
    assert np.max(np.abs(ll - batched) / np.abs(ref)) < TOL


def test_sqrt_real_terms_and_instruments(lib):
    b = W.random_small_batch(951, B=5, n_lo=10, n_hi=80, M=2, J=3)
    rng = np.random.default_rng(952)
    ni = 3
    lab = rng.integers(0, ni, len(b.t_start)).astype(np.int32)
    amp = rng.uniform(0.5, 1.8, (b.n_series, ni))
    off = rng.normal(0.0, 0.4, (b.n_series, ni))
    kinds = ["sho", "real"]
    plan = _plan(lib, b)
    plan.set_term_kinds(kinds)
    # real terms alone
    ll = plan.loglik_sqrt(b.sigma, b.omega0, b.quality, b.jitter).cpu().numpy()
    ref = np.array([kalman.loglik(*_args(b.series(i)), kinds=kinds) for i in range(b.n_series)])
    assert np.max(np.abs(ll - ref) / np.abs(ref)) < TOL
    # and instruments
    plan.set_instruments(lab, ni)
    ll, st = plan.loglik_sqrt(b.sigma, b.omega0, b.quality, b.jitter, amp, off, status=True)
    ll = ll.cpu().numpy()
    assert np.all(st.cpu().numpy() == 0)
    ref = []
    for i in range(b.n_series):
        lo, hi = int(b.offsets[i]), int(b.offsets[i + 1])
        a_n, c_n = kalman.expand_instruments(lab[lo:hi], amp[i], off[i])
        ref.append(kalman.loglik(*_args(b.series(i)), kinds=kinds, amp=a_n, off=c_n))
    ref = np.array(ref)
    batched = plan.loglik_inst(b.sigma, b.omega0, b.quality, b.jitter, amp, off).cpu().numpy()
    print(np.max(np.abs(ll - ref) / np.abs(ref)), np.max(np.abs(ll - batched) / np.abs(ref)))
    assert np.max(np.abs(ll - ref) / np.abs(ref)) < TOL
    assert np.max(np.abs(batched - ref) / np.abs(ref)) < TOL


@pytest.mark.parametrize("instantaneous", [True, False])
def test_sqrt_nearly_noise_free(lib, instantaneous):
    """Measurement errors down to 1e-9 of the signal: the regime the factor
    form is for, against the dense GP in high precision."""
    for noise in (1e-5, 1e-7, 1e-9):
        for omega0 in (0.5, 5.0):
            ts, te, y, yerr, sig, w0, q = CC.smooth(31, 40, noise, omega0, instantaneous)
            Le = exact.loglik(ts, te, y, yerr, sig, w0, q, 0.0, dps=80)
            plan = lib.Plan(np.array([0, len(ts)], dtype=np.int64), ts, te, y, yerr)
            ll = float(plan.loglik_sqrt(sig[None], w0[None], q[None], np.zeros(1), check=True).cpu()[0])
            print(instantaneous, noise, omega0, abs(ll - Le) / abs(Le))
            assert abs(ll - Le) < TOL * abs(Le)
    for seed in (21, 22):
        for noise in (1e-5, 1e-9):
            ts, te, y, yerr, sig, w0, q = CC.two_instruments(seed, 50, noise)
            Le = exact.loglik(ts, te, y, yerr, sig, w0, q, 0.0, dps=80)
            plan = lib.Plan(np.array([0, len(ts)], dtype=np.int64), ts, te, y, yerr)
            ll = float(plan.loglik_sqrt(sig[None], w0[None], q[None], np.zeros(1), check=True).cpu()[0])
            print(seed, noise, abs(ll - Le) / abs(Le))
            assert abs(ll - Le) < TOL * abs(Le)


def test_sqrt_rotations_near_underflow(lib):
    """Rotations of pivot pairs near the bottom of the FP64 range (the
    rotation is scaled by the exponent of its larger entry); without the
    scaling these series are off by 3e-6 ... 1e-4."""
    for seed in range(3):
        ts, te, y, yerr, sig, w0, q = CC.long_gaps(seed)
        ref = kalman.loglik(ts, te, y, yerr, sig, w0, q, 0.0)
        plan = lib.Plan(np.array([0, len(ts)], dtype=np.int64), ts, te, y, yerr)
        ll = float(plan.loglik_sqrt(sig[None], w0[None], q[None], np.zeros(1), check=True).cpu()[0])
        print(seed, abs(ll - ref) / abs(ref))
        assert abs(ll - ref) < TOL * abs(ref)


@pytest.mark.parametrize("case", ["c5_prefix", "m4"])
def test_sqrt_long_series_against_stored_oracle(lib, case):
    """32000 exposures from the generator of the 1e7-exposure workload (three
    terms, up to four overlapping exposures) and a 12000-exposure four-term
    series, against the long-double oracle's stored log-likelihoods
    (tests/golden/kalman_long_scan.json)."""
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "kalman_long_scan.json")) as fh:
        rows = {r["name"]: r for r in json.load(fh)["cases"]}
    r = rows[case]
    b = getattr(W, r["generator"])(**r["kwargs"])
    plan = _plan(lib, b)
    ll = float(plan.loglik_sqrt(b.sigma, b.omega0, b.quality, b.jitter, check=True).cpu()[0])
    rel = abs(ll - r["loglik"]) / abs(r["loglik"])
    print(case, plan.stats()["max_slots"], b.n_terms, rel)
    assert rel < TOL


def test_sqrt_status(lib):
    """A series with invalid hyperparameters is NaN with GP_SSM_EPARAM, the
    others unaffected; an empty series has log-likelihood 0."""
    b = W.random_small_batch(961, B=4, n_lo=5, n_hi=30, M=2, J=2)
    offsets = np.concatenate([b.offsets[:3], b.offsets[2:]])  # series 2 empty
    plan = lib.Plan(offsets, b.t_start, b.t_end, b.y, b.yerr)
    B = len(offsets) - 1
    sig = np.concatenate([b.sigma[:2], b.sigma[1:2], b.sigma[2:]])
    w0 = np.concatenate([b.omega0[:2], b.omega0[1:2], b.omega0[2:]])
    q = np.concatenate([b.quality[:2], b.quality[1:2], b.quality[2:]])
    jit = np.concatenate([b.jitter[:2], b.jitter[1:2], b.jitter[2:]])
    good = plan.loglik_sqrt(sig, w0, q, jit, check=True).cpu().numpy()
    assert good[2] == 0.0
    bad = sig.copy()
    bad[1, 0] = -1.0
    ll, st = plan.loglik_sqrt(bad, w0, q, jit, status=True)
    ll, st = ll.cpu().numpy(), st.cpu().numpy()
    assert st[1] == -3 and np.isnan(ll[1])
    keep = [i for i in range(B) if i != 1]
    assert np.all(st[keep] == 0) and np.array_equal(ll[keep], good[keep])
    with pytest.raises(lib.GpSsmError) as e:
        plan.loglik_sqrt(bad, w0, q, jit, check=True)
    assert e.value.code == -3
    # amplitudes on a plan without instrument labels are refused
    with pytest.raises(lib.GpSsmError) as e:
        plan.loglik_sqrt(sig, w0, q, jit, amp=np.ones(B))
    assert e.value.code == -1


@pytest.mark.parametrize("name", ["grad_1024", "batch_4096"])
def test_sqrt_full_workloads_against_batched(lib, name):
    """The full 1024 x 1e4-exposure gradient workload (three SHO terms, up to
    three overlapping exposures) and the 4096-series batch of uneven length
    (two terms, omega0 up to 1000 / d): every series against the batched
    path."""
    b = getattr(W, name)()
    plan = _plan(lib, b)
    ll_sqrt = plan.loglik_sqrt(b.sigma, b.omega0, b.quality, b.jitter, check=True).cpu().numpy()
    ll = plan.loglik(b.sigma, b.omega0, b.quality, b.jitter, check=True).cpu().numpy()
    rel = np.abs(ll_sqrt - ll) / np.abs(ll)
    print(rel.max(), np.median(rel))
    assert rel.max() < 1e-10


# ---------------------------------------------------------------------------
# the square-root filter split in time (gp_ssm_plan_loglik_sqrt_split)
# ---------------------------------------------------------------------------
SPLITS = (dict(chunk_min=1, chunk_target=1), dict(chunk_min=1, chunk_target=3), dict())


@pytest.mark.parametrize("M,J,T", [(1, 2, 2.0), (2, 3, 2.0), (3, 3, 2.0), (3, 4, 0.4), (4, 2, 2.0)])
def test_sqrt_split_matches_oracle(lib, M, J, T):
    """Chunk summaries in factor form folded per series, at one event per
    chunk, a few and the default chunks: against the oracle and the
    sequential square-root filter."""
    b = W.random_small_batch(970 + 10 * M + J, B=6, n_lo=5, n_hi=70 if T > 1 else 40, M=M, J=J, T=T)
    ref = np.array([kalman.loglik(*_args(b.series(i))) for i in range(b.n_series)])
    seq = None
    for opt in SPLITS:
        plan = _plan(lib, b, **opt)
        ll = plan.loglik_sqrt_split(b.sigma, b.omega0, b.quality, b.jitter, check=True).cpu().numpy()
        if seq is None:
            seq = plan.loglik_sqrt(b.sigma, b.omega0, b.quality, b.jitter, check=True).cpu().numpy()
        rel = np.max(np.abs(ll - ref) / np.abs(ref))
        print(M, J, opt, plan.stats()["n_chunks"], rel, np.max(np.abs(ll - seq) / np.abs(ref)))
        assert rel < TOL
        assert np.max(np.abs(ll - seq) / np.abs(ref)) < 1e-10


def test_sqrt_split_real_terms_and_instruments(lib):
    b = W.random_small_batch(981, B=5, n_lo=10, n_hi=80, M=2, J=3)
    rng = np.random.default_rng(982)
    ni = 3
    lab = rng.integers(0, ni, len(b.t_start)).astype(np.int32)
    amp = rng.uniform(0.5, 1.8, (b.n_series, ni))
    off = rng.normal(0.0, 0.4, (b.n_series, ni))
    kinds = ["sho", "real"]
    ref = []
    for i in range(b.n_series):
        lo, hi = int(b.offsets[i]), int(b.offsets[i + 1])
        a_n, c_n = kalman.expand_instruments(lab[lo:hi], amp[i], off[i])
        ref.append(kalman.loglik(*_args(b.series(i)), kinds=kinds, amp=a_n, off=c_n))
    ref = np.array(ref)
    for opt in SPLITS:
        plan = _plan(lib, b, **opt)
        plan.set_term_kinds(kinds)
        plan.set_instruments(lab, ni)
        ll = plan.loglik_sqrt_split(b.sigma, b.omega0, b.quality, b.jitter, amp, off, check=True).cpu().numpy()
        print(opt, np.max(np.abs(ll - ref) / np.abs(ref)))
        assert np.max(np.abs(ll - ref) / np.abs(ref)) < TOL


def test_sqrt_split_nearly_noise_free(lib):
    """Measurement errors down to 1e-9 of the signal, down to one event per
    chunk (where the covariance-form scan errs by up to 2e-6), against the
    dense GP in high precision."""
    cases = []
    for noise in (1e-5, 1e-7, 1e-9):
        for omega0 in (0.5, 5.0):
            for inst in (True, False):
                cases.append(CC.smooth(31, 40, noise, omega0, inst))
    for seed in (21, 22):
        for noise in (1e-5, 1e-9):
            cases.append(CC.two_instruments(seed, 50, noise))
    worst = 0.0
    for ts, te, y, yerr, sig, w0, q in cases:
        Le = exact.loglik(ts, te, y, yerr, sig, w0, q, 0.0, dps=80)
        for opt in SPLITS:
            plan = lib.Plan(np.array([0, len(ts)], dtype=np.int64), ts, te, y, yerr, **opt)
            ll = float(plan.loglik_sqrt_split(sig[None], w0[None], q[None], np.zeros(1), check=True).cpu()[0])
            worst = max(worst, abs(ll - Le) / abs(Le))
            assert abs(ll - Le) < TOL * abs(Le), (opt, yerr[0], ll, Le)
    print("worst", worst)


@pytest.mark.parametrize("case", ["c5_prefix", "m4"])
def test_sqrt_split_long_series_against_stored_oracle(lib, case):
    with open(os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "kalman_long_scan.json")) as fh:
        rows = {r["name"]: r for r in json.load(fh)["cases"]}
    r = rows[case]
    b = getattr(W, r["generator"])(**r["kwargs"])
    for opt in (dict(chunk_min=1, chunk_target=1), dict()):
        plan = _plan(lib, b, **opt)
        ll = float(plan.loglik_sqrt_split(b.sigma, b.omega0, b.quality, b.jitter, check=True).cpu()[0])
        rel = abs(ll - r["loglik"]) / abs(r["loglik"])
        print(case, opt, plan.stats()["n_chunks"], rel)
        assert rel < TOL


def test_sqrt_split_status_and_full_batch(lib):
    """Invalid hyperparameters and empty series as for the other entry
    points; the full 1024-series gradient workload against the batched
    path."""
    b = W.random_small_batch(991, B=4, n_lo=5, n_hi=30, M=2, J=2)
    offsets = np.concatenate([b.offsets[:3], b.offsets[2:]])
    plan = lib.Plan(offsets, b.t_start, b.t_end, b.y, b.yerr)
    rep = lambda a: np.concatenate([a[:2], a[1:2], a[2:]])
    sig, w0, q, jit = rep(b.sigma), rep(b.omega0), rep(b.quality), rep(b.jitter)
    good = plan.loglik_sqrt_split(sig, w0, q, jit, check=True).cpu().numpy()
    assert good[2] == 0.0
    bad = sig.copy()
    bad[1, 0] = -1.0
    ll, st = plan.loglik_sqrt_split(bad, w0, q, jit, status=True)
    ll, st = ll.cpu().numpy(), st.cpu().numpy()
    assert st[1] == -3 and np.isnan(ll[1])
    keep = [i for i in range(len(good)) if i != 1]
    assert np.all(st[keep] == 0) and np.array_equal(ll[keep], good[keep])
    g = W.grad_1024()
    plan = _plan(lib, g)
    ls = plan.loglik_sqrt_split(g.sigma, g.omega0, g.quality, g.jitter, check=True).cpu().numpy()
    lb = plan.loglik(g.sigma, g.omega0, g.quality, g.jitter, check=True).cpu().numpy()
    print(np.max(np.abs(ls - lb) / np.abs(lb)))
    assert np.max(np.abs(ls - lb) / np.abs(lb)) < 1e-10
