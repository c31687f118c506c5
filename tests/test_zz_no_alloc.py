"""atsfft_execute_batched_noalloc: the batched execute with the library's fixed
device workspace, for callers that cannot allocate.  Its results must be
those of atsfft_execute_batched (with a caller workspace) on the same inputs:
located sets, counts, probed k and statuses identical, values within the
parity tolerance of the precision; checked on two calls in a row, the second
with a smaller batch, and once more after a call the library rejects."""
import numpy as np
import pytest

from paper_1908_02461_amd import synth

from parity_util import VAL_TOL, value_rel_err

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def A():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1908_02461_amd import atsfft

    atsfft.load()
    return atsfft


def _same(plan, out_ref, out_fix, batch, label):
    for i in range(batch):
        r = plan.results(out_ref, i)
        f = plan.results(out_fix, i)
        assert (f["count"], f["khat"], f["status"]) == (r["count"], r["khat"], r["status"]), (label, i)
        assert np.array_equal(f["locs"], r["locs"]), (label, i)
        assert value_rel_err(f["vals"], r["vals"], plan.dtype) < VAL_TOL[plan.dtype], (label, i)


def _signals(n, k, seeds, snr, dtype):
    return np.stack([synth.planted_1d(n, k, s, mag=("uniform", 0.5, 1.0), snr_db=snr, dtype=dtype)[0]
                     for s in seeds])


def test_noalloc_matches_batched_execute(A):
    import torch

    n = 1 << 16
    plan = A.Plan(1, n, "c64", seed=31, max_batch=6)
    assert plan.workspace_size(6) <= A.NOALLOC_WORKSPACE_BYTES
    for step, (batch, k, seeds) in enumerate(((6, 24, range(10, 16)), (2, 8, range(40, 42)))):
        print(f"noalloc call {step}: n={n} batch={batch} k={k}", flush=True)
        x = torch.from_numpy(_signals(n, k, seeds, 30.0, np.complex64)).to("cuda")
        ref = plan.execute_batched(x)
        fix = plan.outputs(batch, x.device)
        plan.execute_noalloc(x, fix)
        torch.cuda.synchronize()
        _same(plan, ref, fix, batch, f"call {step}")


def test_noalloc_two_plans_and_a_rejected_batch(A):
    """A c128 plan, then a shorter c64 one, share the device's array; a batch
    whose workspace exceeds it is refused before anything is launched."""
    import torch

    big = A.Plan(1, 1 << 22, "c64", seed=5, max_batch=64)
    need = big.workspace_size(64)
    assert need > A.NOALLOC_WORKSPACE_BYTES
    x_big = torch.zeros((64, 1 << 22), dtype=torch.complex64, device="cuda")
    with pytest.raises(A.AtsfftError) as e:
        big.execute_noalloc(x_big, big.outputs(64, x_big.device))
    assert e.value.status == A.EINVAL and str(need) in str(e.value)
    del x_big
    for step, (n, dt, batch) in enumerate(((1 << 14, "c128", 3), (1 << 12, "c64", 1))):
        npdt = np.complex128 if dt == "c128" else np.complex64
        snr = None if dt == "c128" else 40.0
        plan = A.Plan(1, n, dt, seed=9 + step, max_batch=batch)
        print(f"noalloc plan {step}: n={n} {dt} batch={batch}", flush=True)
        x = torch.from_numpy(_signals(n, 8, range(70 + 5 * step, 70 + 5 * step + batch), snr, npdt)).to("cuda")
        ref = plan.execute_batched(x)
        fix = plan.outputs(batch, x.device)
        plan.execute_noalloc(x, fix)
        torch.cuda.synchronize()
        _same(plan, ref, fix, batch, f"plan {step}")


def test_noalloc_refuses_allocating_flags(A):
    import torch

    for knobs in (dict(graph=True), dict(profile=True)):
        plan = A.Plan(1, 1 << 12, "c64", seed=1, **knobs)
        x = torch.zeros((1, 1 << 12), dtype=torch.complex64, device="cuda")
        with pytest.raises(A.AtsfftError) as e:
            plan.execute_noalloc(x, plan.outputs(1, x.device))
        assert e.value.status == A.EINVAL
