"""The largest inputs the library accepts: 1D n = 2^30 and 2D N = 2^15
(8 GiB of c64 each).  The oracle cannot run there, so the check is a property
that holds at any size: a noiseless planted spectrum is located exactly
(every planted frequency, nothing of size elsewhere) and its values come back
within the window's leakage."""
import time

import numpy as np
import pytest

from paper_1908_02461_amd import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def A():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1908_02461_amd import atsfft

    atsfft.load()
    return atsfft


def _check(A, plan, x, locs, amps, label):
    import torch

    t0 = time.perf_counter()
    out = plan.execute_batched(x[None])
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    r = plan.results(out, 0)
    print(label, "execute", round(t1 - t0, 3), "s; B*", plan.trace(out["ws"], 0, full=False)["B_star"],
          "located", r["count"], "status", r["status"], flush=True)
    assert not r["status"] & (A.SIG_TRUNCATED | A.SIG_EMPTY)
    idx = np.searchsorted(r["locs"], locs)
    assert np.array_equal(r["locs"][np.clip(idx, 0, len(r["locs"]) - 1)], locs), "a planted frequency is missing"
    err = np.abs(r["vals"][idx] - amps)
    assert err.max() < 1e-3, err.max()
    others = np.delete(np.abs(r["vals"]), idx)
    assert others.size == 0 or others.max() < 1e-3, others.max()


def test_longest_1d(A):
    n, k = 1 << 30, 16
    t0 = time.perf_counter()
    plan = A.Plan(1, n, "c64", seed=3)
    print("plan n=2^30", round(time.perf_counter() - t0, 2), "s", flush=True)
    x, locs, amps = synth.planted_1d_device(n, k, 91, mag=("uniform", 0.5, 1.0))
    _check(A, plan, x, locs, amps, "1D n=2^30")


def test_largest_2d(A):
    N, k = 1 << 15, 16
    t0 = time.perf_counter()
    plan = A.Plan(2, N, "c64", seed=3)
    print("plan N=2^15", round(time.perf_counter() - t0, 2), "s", flush=True)
    x, locs, amps = synth.planted_2d_device(N, k, 92, mag=("uniform", 0.5, 1.0))
    _check(A, plan, x.contiguous(), locs, amps, "2D N=2^15")
