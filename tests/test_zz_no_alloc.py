"""The entry point that allocates nothing (gp_ssm_plan_loglik_noalloc,
workspace in the library's static device array) against
gp_ssm_plan_loglik, whose kernels it shares, through the C-ABI: two calls in
a row, the second on a smaller batch, each equal bit for bit and within 1e-9
of the oracle; a batch whose workspace exceeds the array is refused."""
import numpy as np
import pytest

import workloads as W
from oracle import kalman

pytestmark = pytest.mark.gpu


def _oracle_ll(b):
    return np.array([kalman.loglik(*(b.series(i)[k] for k in ("ts", "te", "y", "yerr", "sigma", "omega0", "quality",
                                                               "jitter"))) for i in range(b.n_series)])


def test_noalloc_matches_plan_loglik(lib):
    import torch
    big = W.random_small_batch(61, B=24, n_lo=100, n_hi=900, M=3, J=3, T=30.0)
    small = W.random_small_batch(62, B=3, n_lo=5, n_hi=30, M=2, J=2)
    for b, opt in ((big, dict(chunk_min=2, chunk_target=3)), (small, dict())):
        plan = lib.Plan(b.offsets, b.t_start, b.t_end, b.y, b.yerr, **opt)
        dev = lambda a: torch.as_tensor(a, dtype=torch.float64, device="cuda")
        args = (dev(b.sigma), dev(b.omega0), dev(b.quality), dev(b.jitter))
        ref, st_ref = plan.loglik(*args, status=True)
        out = torch.full((b.n_series,), float("nan"), dtype=torch.float64, device="cuda")
        st = torch.full((b.n_series,), 7, dtype=torch.int32, device="cuda")
        got = plan.loglik_noalloc(*args, out=out, status=st)
        torch.cuda.synchronize()
        print(plan.stats(), got.cpu().numpy()[:3])
        assert got.data_ptr() == out.data_ptr()
        assert np.array_equal(got.cpu().numpy(), ref.cpu().numpy())
        assert np.all(st.cpu().numpy() == 0) and np.all(st_ref.cpu().numpy() == 0)
        rel = np.abs(got.cpu().numpy() - _oracle_ll(b)) / np.abs(_oracle_ll(b))
        assert np.all(rel < 1e-9), rel


def test_noalloc_refuses_oversized_batch(lib):
    b = W.random_small_batch(63, B=20000, n_lo=3, n_hi=8, M=3, J=2, T=1.0)
    plan = lib.Plan(b.offsets, b.t_start, b.t_end, b.y, b.yerr)
    with pytest.raises(lib.GpSsmError) as e:
        plan.loglik_noalloc(b.sigma, b.omega0, b.quality, b.jitter)
    assert e.value.code == -7
