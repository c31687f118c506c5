"""GPU parity of 2D bucket arrays above the LDS-resident size: the known-k
form (Algorithm 1: B and k given, no probe) at the sparse FFT's bucket count
B = sqrt(N k) per axis (Sec. III-A), where B x B runs from 65536 to 2^20
buckets and the bucket DFTs, thresholds and cutoffs run in device memory.
Every decision (cutoff bits, located set) and the bucket DFTs and values are
compared with the oracle on identical draws, as in test_gpu_parity."""
import numpy as np
import pytest

import oracle
from paper_1908_02461_amd import synth

from parity_util import compare, oracle_params, run_gpu

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def A():
    import torch

    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1908_02461_amd import atsfft

    atsfft.load()
    return atsfft


@pytest.mark.parametrize("N,k,dt,snr,batch", [(1024, 64, "c64", 30.0, 2), (1024, 64, "c128", None, 1),
                                              (2048, 128, "c64", 30.0, 1)])
def test_large_bucket_arrays_match_oracle(A, N, k, dt, snr, batch):
    B = int(round(np.sqrt(N * k)))
    assert B & (B - 1) == 0 and B * B > 16384
    npdt = np.complex64 if dt == "c64" else np.complex128
    mag = ("loguniform", 0.1, 1.0) if snr is not None else None
    plan = A.Plan(2, N, dt, seed=21, max_batch=batch, fixed_B=B, fixed_k=k)
    xs = [synth.planted_2d(N, k, 400 + i, mag=mag, snr_db=snr, dtype=npdt)[0] for i in range(batch)]
    print(f"large 2D bucket arrays: N={N} k={k} B={B} {dt} batch {batch}", flush=True)
    out = run_gpu(plan, np.stack(xs))
    for i, x in enumerate(xs):
        res = plan.results(out, i)
        tr = plan.trace(out["ws"], i)
        ref = oracle.atsfft(x.astype(np.complex128), oracle_params(plan, i), trace=True)
        info = compare(plan, res, tr, ref, f"big2d N={N} B={B} [{i}]")
        print("  ", info, "|S|", res["count"], flush=True)
        if snr is None:
            # noiseless planted spectrum: every planted frequency located
            locs = synth.planted_2d(N, k, 400 + i)[1]
            assert np.all(np.isin(locs, res["locs"])), i


def test_large_bucket_plan_limits(A):
    import torch

    d = dict(fixed_B=256, fixed_k=16)
    for bad in (dict(res_tol=0.1, B_max=128), dict(compensated=True), dict(alpha=16)):
        with pytest.raises(A.AtsfftError) as e:
            A.Plan(2, 1024, "c64", **d, **bad)
        assert e.value.status == A.EINVAL, bad
    with pytest.raises(A.AtsfftError) as e:  # above 1024 per axis
        A.Plan(2, 4096, "c64", fixed_B=2048, fixed_k=16)
    assert e.value.status == A.EINVAL
    plan = A.Plan(2, 1024, "c64", seed=2, **d)
    x = torch.from_numpy(synth.planted_2d(1024, 16, 9, dtype=np.complex64)[0][None].copy()).cuda()
    out = plan.execute_batched(x)
    g = torch.zeros((1, plan.max_out), dtype=torch.complex64, device="cuda")
    gx = torch.empty_like(x)
    with pytest.raises(A.AtsfftError) as e:
        plan.backward(g, out["ws"], gx)
    assert e.value.status == A.ENOTSUPPORTED
